"""Oracle of triplet seeding and helix parameter estimation.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain Python and
numpy in float64, written from the definitions below and sharing nothing
with the GPU library.

The paper (section 2): triplets of spacepoints that can approximately form a
helix are found, and the position and momentum of the track are estimated
at the first spacepoint with the helix model.  It gives no cuts; the
readings:

* spacepoints on the seeding layers (a list of layers ordered outwards)
  take part; a triplet (B, M, T) has its bottom, middle and top on three
  different seeding layers in that order, all of the same event;
* doublet (B, M) and (M, T) cuts, with r the transverse radius and all
  arithmetic in float64 without fused operations: cot = dz / dr with
  |cot| <= COT_MAX; for (B, M) the line's z at r = 0, z_B - r_B cot, within
  Z0_MAX; the azimuth difference within DPHI_MAX, tested as
  dot(xy_1, xy_2) > 0 and |cross(xy_1, xy_2)| <= tan(DPHI_MAX) dot;
* triplet cuts: the circle through the three points in the transverse plane
  has radius >= R_MIN (the helix radius of PT_MIN in the field) and passes
  within D0_MAX of the beam line; |cot_BM - cot_MT| <= DCOT_BASE +
  DCOT_MS (1 + cot_BM^2) (scattering grows with the path length per unit r);
* per middle spacepoint at most KEEP triplets, the smallest (d0, B, T);
  seeds come out by middle spacepoint, then in that order;
* the seed is on B's module: loc = B's local position; phi is the circle's
  tangent at B pointing towards M; theta from the arc length B -> T in the
  transverse plane and dz; q/p = q sin(theta) / pT with pT = kappa Bz R and
  the charge from the turning sense (a positive charge turns clockwise
  seen from +z when Bz > 0); covariance diagonal: 0.2 mm, 0.6 mm, 10 mrad,
  10 mrad and 15 % of q/p (a three-point curvature is good to a few %, with
  tails).
"""
from __future__ import annotations

import math

import numpy as np

KAPPA = 2.99792458e-4            # GeV / (T mm)
COT_MAX = 3.0
Z0_MAX = 200.0                   # mm
DPHI_MAX = 0.12                  # rad
TAN_DPHI = math.tan(DPHI_MAX)
PT_MIN = 0.5                     # GeV
D0_MAX = 1.0                     # mm
DCOT_BASE = 0.01
DCOT_MS = 0.007
KEEP = 2
SEED_SIGMA = (0.2, 0.6, 0.01, 0.01, 0.15)  # loc0, loc1, phi, theta, relative q/p


def r_min(bz):
    return PT_MIN / (KAPPA * abs(bz))


def circle(ax, ay, bx, by, cx, cy):
    """Centre and radius of the circle through three points (float64);
    (nan, nan, inf) for collinear points."""
    d = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    if d == 0.0:
        return math.nan, math.nan, math.inf
    a2, b2, c2 = ax * ax + ay * ay, bx * bx + by * by, cx * cx + cy * cy
    ux = (a2 * (by - cy) + b2 * (cy - ay) + c2 * (ay - by)) / d
    uy = (a2 * (cx - bx) + b2 * (ax - cx) + c2 * (bx - ax)) / d
    rx, ry = ax - ux, ay - uy
    return ux, uy, math.sqrt(rx * rx + ry * ry)


def _doublets(p, q, bottom):
    """Doublet cuts for inner points p [k,3] and outer points q [k,3]
    (elementwise float64: the same operations, in the same order, as the
    scalar definition in the module docstring).  Returns (ok [k], cot [k])."""
    rp = np.sqrt(p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1])
    rq = np.sqrt(q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1])
    dr = rq - rp
    with np.errstate(divide="ignore", invalid="ignore"):
        cot = (q[:, 2] - p[:, 2]) / dr
    ok = (dr > 0.0) & (np.abs(cot) <= COT_MAX)
    if bottom:
        ok &= np.abs(p[:, 2] - rp * cot) <= Z0_MAX
    dot = p[:, 0] * q[:, 0] + p[:, 1] * q[:, 1]
    cross = p[:, 0] * q[:, 1] - p[:, 1] * q[:, 0]
    ok &= (dot > 0.0) & (np.abs(cross) <= TAN_DPHI * dot)
    return ok, cot


def triplets(xyz, layer_index, bz, middles=None):
    """All kept triplets: list of (middle, bottom, top, d0) in output order.
    xyz [n,3] float64 (one event), layer_index [n] (-1: not a seeding
    layer); middles: only these middle spacepoints (default all).  Every
    middle is tested against every other spacepoint of the event (no
    binning)."""
    rmin = r_min(bz)
    n = xyz.shape[0]
    li = np.asarray(layer_index)
    out = []
    for m in (range(n) if middles is None else middles):
        lm = li[m]
        if lm < 0:
            continue
        M = xyz[m]
        jb = np.nonzero((li >= 0) & (li < lm))[0]
        jt = np.nonzero(li > lm)[0]
        okb, cb = _doublets(xyz[jb], np.broadcast_to(M, (len(jb), 3)), True)
        okt, ct = _doublets(np.broadcast_to(M, (len(jt), 3)), xyz[jt], False)
        jb, cb = jb[okb], cb[okb]
        jt, ct = jt[okt], ct[okt]
        if len(jb) == 0 or len(jt) == 0:
            continue
        bb, tt = np.repeat(jb, len(jt)), np.tile(jt, len(jb))
        cbb, ctt = np.repeat(cb, len(jt)), np.tile(ct, len(jb))
        ok = np.abs(cbb - ctt) <= DCOT_BASE + DCOT_MS * (1.0 + cbb * cbb)
        cand = []
        for b, t in zip(bb[ok], tt[ok]):
            B, T = xyz[b], xyz[t]
            ux, uy, R = circle(B[0], B[1], M[0], M[1], T[0], T[1])
            if not R >= rmin:
                continue
            d0 = abs(math.sqrt(ux * ux + uy * uy) - R)
            if not d0 <= D0_MAX:
                continue
            cand.append((d0, int(b), int(t)))
        cand.sort()
        for d0, b, t in cand[:KEEP]:
            out.append((m, b, t, d0))
    return out


def estimate(B, M, T, bz):
    """(phi, theta, q/p) of the helix through B, M, T at B (float64)."""
    ux, uy, R = circle(B[0], B[1], M[0], M[1], T[0], T[1])
    rx, ry = B[0] - ux, B[1] - uy
    tx, ty = -ry / R, rx / R
    if tx * (M[0] - B[0]) + ty * (M[1] - B[1]) < 0.0:
        tx, ty = -tx, -ty
    phi = math.atan2(ty, tx)
    cross = (M[0] - B[0]) * (T[1] - M[1]) - (M[1] - B[1]) * (T[0] - M[0])
    q = 1.0 if (cross < 0.0) == (bz > 0.0) else -1.0
    cx, cy = T[0] - B[0], T[1] - B[1]
    chord = math.sqrt(cx * cx + cy * cy)
    s = 2.0 * R * math.asin(min(1.0, chord / (2.0 * R)))
    theta = math.atan2(s, T[2] - B[2])
    pt = KAPPA * abs(bz) * R
    return phi, theta, q * math.sin(theta) / pt


def seeds(xyz, layer_index, surface, loc, bz):
    """Seeds of one event: dict(bottom, middle, top [k], surface [k],
    params [k,5], cov [k,15])."""
    tr = triplets(xyz, layer_index, bz)
    k = len(tr)
    out = dict(middle=np.array([t[0] for t in tr], np.int64), bottom=np.array([t[1] for t in tr], np.int64),
               top=np.array([t[2] for t in tr], np.int64), surface=np.zeros(k, np.int64),
               params=np.zeros((k, 5)), cov=np.zeros((k, 15)))
    for i, (m, b, t, _) in enumerate(tr):
        phi, theta, qop = estimate(xyz[b], xyz[m], xyz[t], bz)
        out["surface"][i] = surface[b]
        out["params"][i] = (loc[b, 0], loc[b, 1], phi, theta, qop)
        s = SEED_SIGMA
        out["cov"][i, [0, 5, 9, 12, 14]] = (s[0] ** 2, s[1] ** 2, s[2] ** 2, s[3] ** 2, (s[4] * qop) ** 2)
    return out
