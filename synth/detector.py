"""Synthetic silicon tracking detectors (geometry description only).

The paper measures on the Open Data Detector (section 3), which is not
available here; these are stand-ins with the shapes its workloads name:

* ``barrel10``: ten cylindrical barrel layers (r = 30 ... 1000 mm, |z| < 1000
  mm) tiled by flat 20 x 60 mm modules, pixel resolution, no material.
* ``barrel_endcap``: 4 pixel + 4 strip barrel layers and 7 pixel endcap
  disks per side (three rings of 20 x 60 mm modules), 0.01 X0 per module.

Every module is a planar rectangle with a centre ``c`` and three unit row
vectors ``u`` (local axis 0), ``v`` (local axis 1) and ``n = u x v``
(normal).  Each navigation layer carries an envelope: a cylinder of radius
``pos`` with ``lo <= z <= hi`` (barrel) or a plane ``z = pos`` with ``lo <= r
<= hi`` (disk).  The envelope lies on the inner side of every module of its
layer, so an outward-going particle meets it before any of the layer's
modules.

All geometry is built in float64 and then rounded to float32; the float32
values are the detector.  Simulation promotes them back to float64 so that
hits lie exactly on the described planes.

This module holds geometry only: no propagation, fitting or search.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Module size (full lengths, mm) and measurement resolutions (mm).
MODULE_W0 = 20.0
MODULE_W1 = 60.0
PIXEL_SIGMA = (0.015, 0.05)
STRIP_SIGMA = (0.08, 1.2)

BARREL, DISK = 0, 1
PIXEL, STRIP = 0, 1


@dataclass
class Detector:
    name: str
    center: np.ndarray      # (n, 3) float32
    rot: np.ndarray         # (n, 3, 3) float32, rows u, v, n
    half: np.ndarray        # (n, 2) float32 half lengths along u, v
    thick: np.ndarray       # (n,) float32 thickness in radiation lengths
    layer: np.ndarray       # (n,) int32
    kind: np.ndarray        # (n,) int32 PIXEL / STRIP (resolution class)
    layer_type: np.ndarray  # (L,) int32 BARREL / DISK
    layer_pos: np.ndarray   # (L,) float32 radius (barrel) or signed z (disk)
    layer_lo: np.ndarray    # (L,) float32 z_min (barrel) or r_min (disk)
    layer_hi: np.ndarray    # (L,) float32 z_max (barrel) or r_max (disk)
    lattice: list = field(default_factory=list)  # per layer, for the simulator

    @property
    def n_surfaces(self) -> int:
        return int(self.center.shape[0])

    @property
    def n_layers(self) -> int:
        return int(self.layer_type.shape[0])

    def sigma(self) -> np.ndarray:
        """Per-module measurement sigma (n, 2), float32."""
        s = np.where(self.kind[:, None] == PIXEL,
                     np.asarray(PIXEL_SIGMA, np.float32)[None, :],
                     np.asarray(STRIP_SIGMA, np.float32)[None, :])
        return s.astype(np.float32)

    def as_arrays(self) -> dict:
        """Flat, contiguous arrays in the layout both CKF implementations take."""
        return dict(
            center=np.ascontiguousarray(self.center, np.float32),
            rot=np.ascontiguousarray(self.rot.reshape(-1, 9), np.float32),
            half=np.ascontiguousarray(self.half, np.float32),
            thick=np.ascontiguousarray(self.thick, np.float32),
            layer=np.ascontiguousarray(self.layer, np.int32),
            layer_type=np.ascontiguousarray(self.layer_type, np.int32),
            layer_pos=np.ascontiguousarray(self.layer_pos, np.float32),
            layer_lo=np.ascontiguousarray(self.layer_lo, np.float32),
            layer_hi=np.ascontiguousarray(self.layer_hi, np.float32),
        )


class _Builder:
    def __init__(self, name):
        self.name = name
        self.center, self.rot, self.half = [], [], []
        self.thick, self.layer, self.kind = [], [], []
        self.lt, self.lp, self.llo, self.lhi = [], [], [], []
        self.lattice = []
        self.n = 0

    def _add(self, c, u, v, n, thick, layer, kind):
        self.center.append(c)
        self.rot.append(np.stack([u, v, n], axis=-2))
        self.half.append(np.full((c.shape[0], 2), (MODULE_W0 / 2, MODULE_W1 / 2)))
        self.thick.append(np.full(c.shape[0], thick))
        self.layer.append(np.full(c.shape[0], layer))
        self.kind.append(np.full(c.shape[0], kind))
        base = self.n
        self.n += c.shape[0]
        return base

    def barrel(self, R, zhalf, nz, thick, kind):
        """Flat modules tangent to r = R + offset; offsets 1.0 mm by phi
        parity and 0.5 mm by z parity keep overlapping neighbours apart."""
        L = len(self.lt)
        nphi = int(math.ceil(1.05 * math.pi / math.atan(0.5 * MODULE_W0 / (R + 1.5))))
        pitch = (2.0 * zhalf - MODULE_W1) / (nz - 1)
        iz, iphi = np.meshgrid(np.arange(nz), np.arange(nphi), indexing="ij")
        iz, iphi = iz.ravel(), iphi.ravel()
        phic = 2.0 * math.pi * (iphi + 0.5) / nphi
        rm = R + 1.0 * (iphi % 2) + 0.5 * (iz % 2)
        zc = -zhalf + 0.5 * MODULE_W1 + iz * pitch
        c = np.stack([rm * np.cos(phic), rm * np.sin(phic), zc], -1)
        u = np.stack([-np.sin(phic), np.cos(phic), np.zeros_like(phic)], -1)
        v = np.stack([np.zeros_like(phic), np.zeros_like(phic), np.ones_like(phic)], -1)
        n = np.cross(u, v)
        base = self._add(c, u, v, n, thick, L, kind)
        self.lt.append(BARREL)
        self.lp.append(R)
        self.llo.append(-zhalf - 1.0)
        self.lhi.append(zhalf + 1.0)
        self.lattice.append(dict(type=BARREL, base=base, nphi=nphi, nz=nz,
                                 z0=-zhalf + 0.5 * MODULE_W1, pitch=pitch))
        return L

    def disk(self, z, rings, thick, kind):
        """Three rings of radial 20 x 60 mm modules on a disk at signed z.
        Modules sit 1 mm further out by phi parity and 2 mm per ring."""
        L = len(self.lt)
        s = 1.0 if z > 0 else -1.0
        ring_info = []
        for k, (rin, rout) in enumerate(rings):
            nphi = int(math.ceil(1.05 * 2.0 * math.pi * rout / MODULE_W0))
            iphi = np.arange(nphi)
            phic = 2.0 * math.pi * (iphi + 0.5) / nphi
            rc = 0.5 * (rin + rout)
            zm = s * (abs(z) + 1.0 * (iphi % 2) + 2.0 * k)
            c = np.stack([rc * np.cos(phic), rc * np.sin(phic), zm], -1)
            v = np.stack([np.cos(phic), np.sin(phic), np.zeros_like(phic)], -1)
            n = np.tile(np.array([0.0, 0.0, s]), (nphi, 1))
            u = np.cross(v, n)
            base = self._add(c, u, v, n, thick, L, kind)
            ring_info.append(dict(base=base, nphi=nphi, rin=rin, rout=rout))
        self.lt.append(DISK)
        self.lp.append(z)
        self.llo.append(rings[0][0] - 5.0)
        self.lhi.append(rings[-1][1] + 1.0)
        self.lattice.append(dict(type=DISK, side=s, rings=ring_info))
        return L

    def build(self) -> Detector:
        f32 = np.float32
        return Detector(
            name=self.name,
            center=np.concatenate(self.center).astype(f32),
            rot=np.concatenate(self.rot).astype(f32),
            half=np.concatenate(self.half).astype(f32),
            thick=np.concatenate(self.thick).astype(f32),
            layer=np.concatenate(self.layer).astype(np.int32),
            kind=np.concatenate(self.kind).astype(np.int32),
            layer_type=np.asarray(self.lt, np.int32),
            layer_pos=np.asarray(self.lp, f32),
            layer_lo=np.asarray(self.llo, f32),
            layer_hi=np.asarray(self.lhi, f32),
            lattice=self.lattice,
        )


def barrel10(thick: float = 0.0) -> Detector:
    """Ten barrel layers, |z| < 1000 mm, pixel modules (the tiny oracle event)."""
    b = _Builder("barrel10")
    for R in (30, 70, 120, 180, 260, 360, 500, 660, 820, 1000):
        b.barrel(float(R), 1000.0, 36, thick, PIXEL)
    return b.build()


DISK_Z = (600.0, 700.0, 820.0, 960.0, 1120.0, 1300.0, 1500.0)
DISK_RINGS = ((30.0, 90.0), (85.0, 145.0), (140.0, 200.0))


def barrel_endcap(thick: float = 0.01) -> Detector:
    """4 pixel barrel layers (|z| < 500), 4 strip barrel layers (|z| < 1000)
    and 7 pixel disks per side: the dense-event detector."""
    b = _Builder("barrel_endcap")
    for R in (30, 70, 120, 180):
        b.barrel(float(R), 500.0, 18, thick, PIXEL)
    for R in (260, 360, 500, 660):
        b.barrel(float(R), 1000.0, 36, thick, STRIP)
    for z in DISK_Z:
        b.disk(z, DISK_RINGS, thick, PIXEL)
    for z in DISK_Z:
        b.disk(-z, DISK_RINGS, thick, PIXEL)
    return b.build()
