"""Truth trajectories in a non-uniform magnetic field (a field map study).

In a field that is not uniform a charged particle's path is no helix, so
its module crossings have no closed form.  Here every particle is
integrated numerically, all particles together: the classical fourth-order
Runge-Kutta method in FP64 on (r, T) in path length s, dr/ds = T,
dT/ds = kappa (q/p) T x B(r), with a fixed step of ``step`` mm and the
analytic field (not a grid).  Within each step the path is the cubic
Hermite curve through the two end states (position error ~ step^4 / R^3,
below 1e-7 mm for step = 10 mm and R >= 0.8 m); a module is crossed where
that curve changes sides of the module plane inside its bounds (root by
bisection to 1e-12 of the step), and the first crossing of the step ends
it: the crossing is recorded (position on the plane, unit tangent there),
the multiple-scattering kick of the module is applied, and the integration
restarts from it.  A particle stops after half a turn in the transverse
plane (as the closed-form simulator), beyond the detector, after a path of
``path_max`` mm, or after ``max_cross`` crossings.

With a uniform axial field this reproduces the closed-form helix
simulator's crossings (tests/test_synth.py).  This module is a simulator:
it holds no propagation, search or fitting arithmetic of the track finders.
"""
from __future__ import annotations

import math

import numpy as np

from .detector import BARREL, Detector

C_LIGHT = 2.99792458e-4  # GeV / (T mm) per unit charge


def _bands(det: Detector):
    """Per layer the range of the module planes in the layer's coordinate:
    radius for barrels (plane distance to the axis up to the corner radius),
    z for disks; 0.5 mm of slack."""
    out = []
    c = det.center.astype(np.float64)
    n = det.rot[:, 2].astype(np.float64)
    h = det.half.astype(np.float64)
    for L in range(det.n_layers):
        m = det.layer == L
        if det.layer_type[L] == BARREL:
            d = np.abs(np.einsum("ki,ki->k", n[m], c[m]))
            r_hi = np.sqrt(d * d + h[m, 0] ** 2 + 0.0)
            out.append((float(d.min()) - 0.5, float(r_hi.max()) + 0.5))
        else:
            out.append((float(c[m, 2].min()) - 0.5, float(c[m, 2].max()) + 0.5))
    return out


def _rk4(field, kq, r, T, h):
    """One classical RK4 step of length h for dr/ds = T, dT/ds = kq T x B(r)."""
    def f(rr, TT):
        return TT, kq[:, None] * np.cross(TT, field(rr))
    k1r, k1t = f(r, T)
    k2r, k2t = f(r + 0.5 * h[:, None] * k1r, T + 0.5 * h[:, None] * k1t)
    k3r, k3t = f(r + 0.5 * h[:, None] * k2r, T + 0.5 * h[:, None] * k2t)
    k4r, k4t = f(r + h[:, None] * k3r, T + h[:, None] * k3t)
    r1 = r + h[:, None] / 6.0 * (k1r + 2 * k2r + 2 * k3r + k4r)
    T1 = T + h[:, None] / 6.0 * (k1t + 2 * k2t + 2 * k3t + k4t)
    return r1, T1 / np.linalg.norm(T1, axis=1)[:, None]


def _hermite(r0, T0, r1, T1, h, t):
    """Point and unit tangent at parameter t of the cubic Hermite curve with
    end points r0, r1 and end derivatives h T0, h T1 (shapes broadcast)."""
    t2, t3 = t * t, t * t * t
    h00, h10, h01, h11 = 2 * t3 - 3 * t2 + 1, t3 - 2 * t2 + t, -2 * t3 + 3 * t2, t3 - t2
    d00, d10, d01, d11 = 6 * t2 - 6 * t, 3 * t2 - 4 * t + 1, -6 * t2 + 6 * t, 3 * t2 - 2 * t
    hh = h[..., None]
    X = h00[..., None] * r0 + (h10[..., None] * hh) * T0 + h01[..., None] * r1 + (h11[..., None] * hh) * T1
    D = d00[..., None] * r0 + (d10[..., None] * hh) * T0 + d01[..., None] * r1 + (d11[..., None] * hh) * T1
    return X, D / np.linalg.norm(D, axis=-1, keepdims=True)


def simulate_field(det: Detector, vtx, mom, q, field, rng, material=True, max_cross=80, step=10.0,
                   path_max=4000.0):
    """Module crossings of particles (vertex vtx [N, 3], momentum mom [N, 3]
    GeV, charge q [N]) in the field ``field(points [M, 3]) -> B [M, 3]``
    (tesla).  Returns a dict of arrays in the closed-form simulator's Truth
    layout (particle, surface, loc, pos, dir, qop, order), unsorted."""
    from .events import _lattice_candidates, highland, MUON_MASS
    N = vtx.shape[0]
    pos = vtx.astype(np.float64).copy()
    p = np.linalg.norm(mom, axis=1)
    T = mom / p[:, None]
    qop = q / p
    kq = C_LIGHT * qop
    cur = np.full(N, -1, np.int64)
    count = np.zeros(N, np.int64)
    turned = np.zeros(N)
    path = np.zeros(N)
    alive = np.ones(N, bool)
    bands = _bands(det)
    # beyond these a particle on its first half turn crosses nothing more
    r_out = max(hi for (lo, hi), t in zip(bands, det.layer_type) if t == BARREL) + 5.0
    z_out = max(float(np.max(np.abs(det.center[:, 2]))) + float(np.max(det.half)), 0.0) + 5.0
    c_all = det.center.astype(np.float64)
    R_all = det.rot.astype(np.float64)
    h_all = det.half.astype(np.float64)
    rec = {k: [] for k in ("particle", "surface", "loc", "pos", "dir", "qop", "order")}
    while alive.any():
        idx = np.nonzero(alive)[0]
        r0, T0 = pos[idx], T[idx]
        h = np.full(idx.size, step)
        r1, T1 = _rk4(field, kq[idx], r0, T0, h)
        rho0, rho1 = np.hypot(r0[:, 0], r0[:, 1]), np.hypot(r1[:, 0], r1[:, 1])
        hits_p, hits_t, hits_m = [], [], []
        for L in range(det.n_layers):
            lo, hi = bands[L]
            if det.layer_type[L] == BARREL:
                w0, w1 = np.minimum(rho0, rho1) - 1.0, np.maximum(rho0, rho1) + 1.0
            else:
                w0, w1 = np.minimum(r0[:, 2], r1[:, 2]) - 1.0, np.maximum(r0[:, 2], r1[:, 2]) + 1.0
            sel = np.nonzero((w1 >= lo) & (w0 <= hi))[0]
            if sel.size == 0:
                continue
            mid = 0.5 * (r0[sel] + r1[sel])
            cand = _lattice_candidates(det, L, mid)  # [M, k]
            cand = np.where(cand == cur[idx[sel]][:, None], -1, cand)
            cs = np.maximum(cand, 0)
            nrm = R_all[cs, 2]
            cc = c_all[cs]
            f0 = np.einsum("mki,mki->mk", nrm, r0[sel][:, None, :] - cc)
            f1 = np.einsum("mki,mki->mk", nrm, r1[sel][:, None, :] - cc)
            ok = (cand >= 0) & (f0 * f1 <= 0.0) & ~((f0 == 0.0) & (f1 == 0.0))
            if not ok.any():
                continue
            mi, ki = np.nonzero(ok)
            a = np.zeros(mi.size)
            b = np.ones(mi.size)
            ra0, ta0, ra1, ta1 = r0[sel][mi], T0[sel][mi], r1[sel][mi], T1[sel][mi]
            ha = h[sel][mi]
            nn, ccc, fa = nrm[mi, ki], cc[mi, ki], f0[mi, ki]
            for _ in range(42):  # bisection on the side of the plane
                t = 0.5 * (a + b)
                X, _ = _hermite(ra0, ta0, ra1, ta1, ha, t)
                ft = np.einsum("ki,ki->k", nn, X - ccc)
                same = (ft * fa) > 0.0
                a = np.where(same, t, a)
                b = np.where(same, b, t)
            t = 0.5 * (a + b)
            X, _ = _hermite(ra0, ta0, ra1, ta1, ha, t)
            m_id = cs[mi, ki]
            d = X - c_all[m_id]
            l0 = np.einsum("ki,ki->k", R_all[m_id, 0], d)
            l1 = np.einsum("ki,ki->k", R_all[m_id, 1], d)
            inside = (np.abs(l0) <= h_all[m_id, 0]) & (np.abs(l1) <= h_all[m_id, 1])
            hits_p.append(sel[mi][inside])
            hits_t.append(t[inside])
            hits_m.append(m_id[inside])
        # the first crossing of the step (smallest t, ties by module id)
        best_t = np.full(idx.size, np.inf)
        best_m = np.full(idx.size, -1, np.int64)
        if hits_p:
            hp, ht, hm = np.concatenate(hits_p), np.concatenate(hits_t), np.concatenate(hits_m)
            if hp.size:
                o = np.lexsort((hm, ht, hp))
                first = o[np.r_[True, hp[o][1:] != hp[o][:-1]]]
                best_t[hp[first]], best_m[hp[first]] = ht[first], hm[first]
        hit = best_m >= 0
        # particles without a crossing in this step move to its end
        nh = ~hit
        gi = idx[nh]
        pos[gi], T[gi] = r1[nh], T1[nh]
        path[gi] += step
        ang = np.abs(np.arctan2(T0[nh, 0] * T1[nh, 1] - T0[nh, 1] * T1[nh, 0],
                                T0[nh, 0] * T1[nh, 0] + T0[nh, 1] * T1[nh, 1]))
        turned[gi] += ang
        if hit.any():
            m = np.nonzero(hit)[0]
            gi = idx[m]
            t = best_t[m]
            surf = best_m[m]
            X, D = _hermite(r0[m], T0[m], r1[m], T1[m], h[m], t)
            d = X - c_all[surf]
            rec["particle"].append(gi)
            rec["surface"].append(surf)
            rec["loc"].append(np.stack([np.einsum("ki,ki->k", R_all[surf, 0], d),
                                        np.einsum("ki,ki->k", R_all[surf, 1], d)], -1))
            rec["pos"].append(X)
            rec["dir"].append(D)
            rec["qop"].append(qop[gi])
            rec["order"].append(count[gi].copy())
            count[gi] += 1
            path[gi] += t * step
            turned[gi] += np.abs(np.arctan2(T0[m, 0] * D[:, 1] - T0[m, 1] * D[:, 0],
                                            T0[m, 0] * D[:, 0] + T0[m, 1] * D[:, 1]))
            if material:
                th = det.thick[surf].astype(np.float64)
                cosa = np.abs(np.einsum("ki,ki->k", R_all[surf, 2], D))
                x = th / np.maximum(cosa, 1e-12)
                th0 = np.where(th > 0, highland(1.0 / np.abs(qop[gi]), MUON_MASS, np.maximum(x, 1e-30)), 0.0)
                theta0 = np.arccos(np.clip(D[:, 2], -1.0, 1.0))
                theta = theta0 + th0 * rng.standard_normal(gi.size)
                phi = np.arctan2(D[:, 1], D[:, 0]) + th0 * rng.standard_normal(gi.size) / np.sin(theta0)
                D = np.stack([np.cos(phi) * np.sin(theta), np.sin(phi) * np.sin(theta), np.cos(theta)], -1)
            pos[gi], T[gi], cur[gi] = X, D, surf
        rho = np.hypot(pos[idx, 0], pos[idx, 1])
        gone = ((turned[idx] >= math.pi) | (path[idx] >= path_max) | (rho > r_out) |
                (np.abs(pos[idx, 2]) > z_out) | (count[idx] >= max_cross))
        alive[idx[gone]] = False
    cat = {k: (np.concatenate(v) if v else np.zeros((0,) + ((2,) if k == "loc" else (3,) if k in ("pos", "dir") else ())))
           for k, v in rec.items()}
    return cat
