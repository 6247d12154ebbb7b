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
