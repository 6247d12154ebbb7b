"""Magnetic-field maps on a regular (r, z) grid (inputs, FP32 values).

solenoid_map(): B_z(z) = 0.5 + 1.5 cos^2(pi z / 6000) T for |z| <= 3000 mm
(0.5 T beyond), falling from 2.0 T at the centre towards 0.5 T at |z| = 3 m;
B_r(r, z) = -(r / 2) dB_z/dz, which makes div B = 0 exactly (B_z does not
depend on r).  Grid r in [0, 1200] mm, z in [-3000, 3000] mm at 5 mm
(241 x 1201 nodes); the grid, interpolated bilinearly with clamped
coordinates, is the field's definition for both track finders.

linear_map(): B_z = b0 + g z, B_r = -(r / 2) g - linear in r and z, so
bilinear interpolation reproduces it exactly (a test field).

Layout: values[iz, ir, 0] = B_r, values[iz, ir, 1] = B_z at r0 + ir*dr,
z0 + iz*dz.
"""
from __future__ import annotations

import numpy as np


def _grid(r_max, z_max, step):
    nr = int(round(r_max / step)) + 1
    nz = int(round(2 * z_max / step)) + 1
    r = np.arange(nr) * step
    z = -z_max + np.arange(nz) * step
    return r, z


def solenoid_bz(z):
    z = np.asarray(z, np.float64)
    c = np.cos(np.pi * z / 6000.0)
    return np.where(np.abs(z) <= 3000.0, 0.5 + 1.5 * c * c, 0.5)


def solenoid_dbz_dz(z):
    z = np.asarray(z, np.float64)
    # d/dz of 1.5 cos^2(pi z / 6000) = -1.5 (pi / 6000) sin(pi z / 3000)
    return np.where(np.abs(z) <= 3000.0, -1.5 * (np.pi / 6000.0) * np.sin(np.pi * z / 3000.0), 0.0)


def solenoid_field(p):
    """Analytic field (T) at points p [..., 3] (mm)."""
    p = np.asarray(p, np.float64)
    r = np.hypot(p[..., 0], p[..., 1])
    br = -0.5 * r * solenoid_dbz_dz(p[..., 2])
    with np.errstate(invalid="ignore", divide="ignore"):
        cx = np.where(r > 0, p[..., 0] / np.where(r > 0, r, 1), 0.0)
        sy = np.where(r > 0, p[..., 1] / np.where(r > 0, r, 1), 0.0)
    return np.stack([br * cx, br * sy, solenoid_bz(p[..., 2])], axis=-1)


def solenoid_map(r_max=1200.0, z_max=3000.0, step=5.0) -> dict:
    r, z = _grid(r_max, z_max, step)
    R, Z = np.meshgrid(r, z)  # [nz, nr]
    vals = np.stack([-0.5 * R * solenoid_dbz_dz(Z), solenoid_bz(Z)], axis=-1).astype(np.float32)
    return dict(map=np.ascontiguousarray(vals), nr=r.size, nz=z.size, r0=0.0, z0=-z_max, dr=step, dz=step)


def linear_map(b0=2.0, g=-2e-4, r_max=1200.0, z_max=3000.0, step=5.0) -> dict:
    r, z = _grid(r_max, z_max, step)
    R, Z = np.meshgrid(r, z)
    vals = np.stack([-0.5 * R * g, b0 + g * Z], axis=-1).astype(np.float32)
    return dict(map=np.ascontiguousarray(vals), nr=r.size, nz=z.size, r0=0.0, z0=-z_max, dr=step, dz=step)
