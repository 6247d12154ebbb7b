"""Track-by-track comparison of two track finders' outputs (seed-ordered
CSR dicts), with the parameter tolerance of the parity tests:
|a - b| <= 1e-4 * max(|ref|, s) with s = 10 mm (loc0), 30 mm (loc1), 1 rad
(phi, wrap-aware), 1 rad (theta), |q/p| (q/p); covariance diagonals 1e-4
relative, correlation coefficients 1e-4 absolute."""
import math

import numpy as np

PARAM_SCALE = np.array([10.0, 30.0, 1.0, 1.0, 0.0])
DIAG = [0, 5, 9, 12, 14]


def unpack_cov(c15):
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i, 5):
            M[i, j] = M[j, i] = c15[k]
            k += 1
    return M


def compare(ref, got):
    """Returns (identical, mismatches [(seed, kind)], extra seeds, worst
    parameter error per quantity, worst covariance error)."""
    ref_by_seed = {int(ref["seed"][t]): t for t in range(ref["n_tracks"])}
    got_by_seed = {int(got["seed"][t]): t for t in range(got["n_tracks"])}
    same = 0
    worst = np.zeros(5)
    cov_worst = 0.0
    mism = []
    for s, t in ref_by_seed.items():
        a = ref["meas"][ref["offsets"][t]:ref["offsets"][t + 1]]
        u = got_by_seed.get(s)
        if u is None:
            mism.append((s, "missing"))
            continue
        b = got["meas"][got["offsets"][u]:got["offsets"][u + 1]]
        if not np.array_equal(a, b):
            mism.append((s, "pattern"))
            continue
        same += 1
        pr, pg = ref["params"][t], got["params"][u]
        d = pg - pr
        d[2] = (d[2] + math.pi) % (2 * math.pi) - math.pi
        scale = np.maximum(np.abs(pr), PARAM_SCALE)
        scale[4] = abs(pr[4])
        worst = np.maximum(worst, np.abs(d) / scale)
        cr, cg = ref["cov"][t], got["cov"][u]
        cov_worst = max(cov_worst, np.max(np.abs(cg[DIAG] - cr[DIAG]) / cr[DIAG]))
        Mr, Mg = unpack_cov(cr), unpack_cov(cg)
        dr, dg = np.sqrt(np.diag(Mr)), np.sqrt(np.diag(Mg))
        cov_worst = max(cov_worst, np.max(np.abs(Mg / np.outer(dg, dg) - Mr / np.outer(dr, dr))))
    extra = [s for s in got_by_seed if s not in ref_by_seed]
    return same, mism, extra, worst, cov_worst


def decoy_event():
    """The enumeration input: four pixel barrel layers, a tiny event whose
    every hit has up to two decoy hits on the same module (Gaussian, 3 sigma
    of the resolution), and every 17th seed.  Returns (detector, event,
    seed indices kept)."""
    from synth import make_event
    from synth.detector import _Builder, PIXEL
    b = _Builder("four")
    for R in (30.0, 70.0, 120.0, 180.0):
        b.barrel(R, 300.0, 11, 0.0, PIXEL)
    det = b.build()
    ev = make_event(det, 7, kind="tiny")
    rng = np.random.default_rng(1)
    keep = np.arange(0, ev.n_seeds, 17)
    loc, var, surf, part = [], [], [], []
    for s in range(det.n_surfaces):
        for i in range(ev.offsets[s], ev.offsets[s + 1]):
            loc.append(ev.loc[i]); var.append(ev.var[i]); surf.append(s); part.append(ev.meas_particle[i])
            for _ in range(rng.integers(0, 3)):
                loc.append(ev.loc[i] + rng.normal(0, 3.0, 2) * np.sqrt(ev.var[i]))
                var.append(ev.var[i]); surf.append(s); part.append(-1)
    surf = np.asarray(surf)
    ev.loc, ev.var = np.asarray(loc, np.float32), np.asarray(var, np.float32)
    ev.meas_particle = np.asarray(part)
    ev.offsets = np.r_[0, np.cumsum(np.bincount(surf, minlength=det.n_surfaces))].astype(np.int32)
    return det, ev, keep
