"""Pins of the oracle's track finding as a whole (paper section 2: navigation
to intersected modules, chi2 gating, branching; section 3.1: validation
through matching and efficiency) against the simulation's truth, pull
statistics, an independent depth-first enumeration and invariances."""
import math

import numpy as np
import pytest

from conftest import double_matched
from synth import make_event

PACKED_DIAG = (0, 5, 9, 12, 14)


def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


@pytest.mark.parametrize("which", ["barrel", "dense_vacuum"])
def test_navigator_follows_truth(oracle_lib, det_barrel, det_dense_vacuum, which):
    """Without material the truth trajectory is an exact helix; started from
    the true parameters, the navigator crosses exactly the modules the
    simulator's closed-form crossing search found, in the same order."""
    det = det_barrel if which == "barrel" else det_dense_vacuum
    ev = make_event(det, 21, kind="tiny" if which == "barrel" else "pileup", mu=4, smear_seeds=False)
    inp = oracle_lib.Inputs(det.as_arrays(), (0, 0, 2.0))
    tr = ev.truth
    same = 0
    for k in range(ev.n_seeds):
        p = ev.seed_particle[k]
        truth = tr.surface[tr.particle == p]
        vis, cr, _ = oracle_lib.trace(inp, ev.seed_surface[k], ev.seed_truth[k], material_on=0)
        got = vis[cr == 1]
        same += int(list(got) == list(truth[1:]))
    assert same >= 0.995 * ev.n_seeds, (same, ev.n_seeds)


def _pulls(oracle_lib, det, events, **cfg):
    inp = oracle_lib.Inputs(det.as_arrays(), (0, 0, 2.0))
    pulls, chi2n = [], []
    for ev in events:
        inp.set_event(ev)
        out = oracle_lib.ckf_find(inp, n_threads=4, **cfg)
        tr = ev.truth
        for t in range(out["n_tracks"]):
            s = out["seed"][t]
            ids = out["meas"][out["offsets"][t]:out["offsets"][t + 1]]
            p = ev.seed_particle[s]
            if not np.all(ev.meas_particle[ids] == p):
                continue
            surf = out["last_surface"][t]
            row = np.nonzero((tr.particle == p) & (tr.surface == surf))[0]
            if row.size != 1:
                continue
            r = row[0]
            d = tr.dir[r]
            truth = np.array([tr.loc[r, 0], tr.loc[r, 1], math.atan2(d[1], d[0]),
                              math.acos(np.clip(d[2], -1, 1)), tr.qop[r]])
            fit = out["params"][t]
            diff = fit - truth
            diff[2] = _wrap(diff[2])
            sig = np.sqrt(out["cov"][t][list(PACKED_DIAG)])
            pulls.append(diff / sig)
            chi2n.append(out["chi2"][t] / (2 * len(ids)))
    return np.array(pulls), np.array(chi2n)


def test_pulls_unit_width_no_material(oracle_lib, det_barrel):
    """Exact helices, Gaussian hits, consistent seed covariance: the filtered
    parameters at the last measurement have unit-width, zero-mean pulls and
    the chi2 sum per measured degree of freedom averages 1."""
    events = [make_event(det_barrel, 100 + i, kind="tiny") for i in range(25)]
    P, X = _pulls(oracle_lib, det_barrel, events, material_on=0)
    assert P.shape[0] > 2000
    np.testing.assert_allclose(P.mean(0), 0.0, atol=0.08)
    np.testing.assert_allclose(P.std(0), 1.0, atol=0.05)
    assert X.mean() == pytest.approx(1.0, abs=0.03)


def test_pulls_unit_width_with_scattering(oracle_lib, det_dense):
    """With 1 % X0 per module the simulator kicks each particle by Highland-
    width angles; the filter's scattering noise must keep the pulls at unit
    width (a wrong noise term widens or narrows them)."""
    events = [make_event(det_dense, 300 + i, mu=20) for i in range(3)]
    P, X = _pulls(oracle_lib, det_dense, events)
    assert P.shape[0] > 2000
    np.testing.assert_allclose(P.mean(0), 0.0, atol=0.08)
    np.testing.assert_allclose(P.std(0), 1.0, atol=0.06)
    assert X.mean() == pytest.approx(1.0, abs=0.04)


def test_true_hit_chi2_is_chi2_two_dof(oracle_lib, det_barrel):
    """The gate's chi2 (paper section 2: from the predicted covariance and
    the residual) of a particle's own hit, predicted by propagating the
    filtered state along the particle's true crossings: without material the
    residual is Gaussian with covariance S = H C H^T + V, so the values follow
    the chi-square law with 2 degrees of freedom, CDF 1 - exp(-x/2).  The
    Kolmogorov-Smirnov distance stays below its 1 % critical value 1.63/sqrt(n)
    (a variance 20 % off moves it to about four times that), the mean is 2."""
    x2 = []
    inp = oracle_lib.Inputs(det_barrel.as_arrays(), (0, 0, 2.0))
    for i in range(6):
        ev = make_event(det_barrel, 700 + i, kind="tiny")
        inp.set_event(ev)
        tr = ev.truth
        for k in range(ev.n_seeds):
            p = ev.seed_particle[k]
            path = tr.surface[tr.particle == p]
            s, x, C = int(ev.seed_surface[k]), ev.seed_params[k].copy(), ev.seed_cov[k].copy()
            assert path[0] == s
            for j, m in enumerate(path):
                if j > 0:
                    res = oracle_lib.propagate(inp, s, x, C, int(m), material_on=0)
                    assert res is not None
                    x, C, _, _ = res
                    s = int(m)
                mine = [q for q in range(ev.offsets[s], ev.offsets[s + 1]) if ev.meas_particle[q] == p]
                if len(mine) != 1:
                    continue
                q = mine[0]
                x, C, c2 = oracle_lib.kf_update(x, C, ev.loc[q].astype(float), ev.var[q].astype(float))
                if j > 0:
                    x2.append(c2)
    v = np.sort(np.array(x2))
    n = len(v)
    assert n > 5000
    F = 1.0 - np.exp(-v / 2.0)
    D = max(np.max(np.arange(1, n + 1) / n - F), np.max(F - np.arange(n) / n))
    assert D < 1.63 / math.sqrt(n), D
    assert v.mean() == pytest.approx(2.0, abs=6 * 2.0 / math.sqrt(n))


def test_efficiency_tiny_event(oracle_lib, det_barrel):
    """Isolated 1-10 GeV muons, 99 % hit efficiency: at least 98 % of seeds
    give a double-matched track (paper section 3.1 definition)."""
    ev = make_event(det_barrel, 1, kind="tiny")
    inp = oracle_lib.Inputs(det_barrel.as_arrays(), (0, 0, 2.0), ev)
    out = oracle_lib.ckf_find(inp, n_threads=4, material_on=0)
    ok = 0
    for t in range(out["n_tracks"]):
        ids = out["meas"][out["offsets"][t]:out["offsets"][t + 1]]
        ok += double_matched(ev, ids, ev.seed_particle[out["seed"][t]])
    assert ok >= 0.98 * ev.n_seeds


# ---------------------------------------------------------------------------
# Independent depth-first enumeration of the same search (no pruning, every
# passing measurement branches): the oracle's finished set must equal it.

def _dfs_all(oracle_lib, inp, ev, k, cfg):
    """Recursive enumeration of one seed's tree using only the oracle's
    navigator, propagator and single update; gating, branching, holes, step
    budget and termination are re-implemented here."""
    from oracle import unpack_cov, pack_cov
    out = []
    chi2_max, max_holes, max_steps = cfg["chi2_max"], cfg["max_holes"], cfg["max_steps"]
    ev_i = ev.seed_event[k]

    def search(c):
        row = ev_i * ev.n_surfaces + c["surface"]
        C = unpack_cov(c["cov"])
        acc = []
        for i in range(ev.offsets[row], ev.offsets[row + 1]):
            r = ev.loc[i].astype(float) - c["p"][:2]
            S = C[:2, :2] + np.diag(ev.var[i].astype(float))
            x2 = float(r @ np.linalg.solve(S, r))
            if x2 < chi2_max:
                acc.append((x2, i))
        acc.sort()
        if not acc:
            c = dict(c, holes=c["holes"] + 1)
            if c["holes"] > max_holes:
                out.append(c)
            else:
                advance(c)
            return
        for x2, i in acc:
            po, co, _ = oracle_lib.kf_update(c["p"], c["cov"], ev.loc[i].astype(float), ev.var[i].astype(float))
            advance(dict(c, p=po, cov=co, n=c["n"] + 1, chi2=c["chi2"] + x2, ids=c["ids"] + [i]))

    def advance(c):
        c = dict(c, step=c["step"] + 1)
        if c["step"] >= max_steps:
            out.append(c)
            return
        lst = list(c["list"])
        if not lst:
            L, lst = oracle_lib.navigate(inp, c["surface"], c["p"], c["mask"], c["path"], **cfg)
            if L < 0:
                out.append(c)
                return
            c = dict(c, mask=c["mask"] | (1 << L), list=lst)
            if not lst:
                advance(c)
                return
        m = lst.pop(0)
        res = oracle_lib.propagate(inp, c["surface"], c["p"], c["cov"], m, **cfg)
        if res is None:
            return
        po, co, _, path = res
        c = dict(c, surface=m, p=po, cov=co, list=lst, path=c["path"] + path)
        h = inp.keep[0]["half"][m]
        if not (abs(po[0]) <= h[0] and abs(po[1]) <= h[1]):
            advance(c)
            return
        search(c)

    root = dict(surface=int(ev.seed_surface[k]), p=ev.seed_params[k].copy(), cov=ev.seed_cov[k].copy(),
                n=0, chi2=0.0, holes=0, ids=[], mask=1 << int(inp.keep[0]["layer"][ev.seed_surface[k]]),
                list=oracle_lib.seed_list(inp, ev.seed_surface[k], ev.seed_params[k], **cfg),
                path=0.0, step=0)
    search(root)
    return out


def test_ckf_equals_exhaustive_enumeration(oracle_lib):
    """Four pixel layers crowded with decoy hits near every true hit, all
    branches kept, no pruning: the oracle's finished candidates equal the
    depth-first enumeration of all gated sequences."""
    from parity_util import decoy_event
    det, ev, keep = decoy_event()
    cfg = dict(oracle_lib.DEFAULT_CONFIG, branches_per_surface=0, max_live_per_seed=0, tracks_per_seed=0,
               min_meas=0, material_on=0, max_steps=12, step_tol=1e-6)
    inp = oracle_lib.Inputs(det.as_arrays(), (0, 0, 2.0))
    inp.set_event(ev, seeds=keep)
    got = oracle_lib.ckf_find(inp, n_threads=1, **cfg)
    inp.set_event(ev)
    n_multi = 0
    for j, k in enumerate(keep):
        mine = [t for t in range(got["n_tracks"]) if got["seed"][t] == j]
        gseq = sorted((tuple(int(i) for i in got["meas"][got["offsets"][t]:got["offsets"][t + 1]]),
                       got["chi2"][t]) for t in mine)
        ref = _dfs_all(oracle_lib, inp, ev, k, cfg)
        rseq = sorted((tuple(c["ids"]), c["chi2"]) for c in ref)
        assert [g[0] for g in gseq] == [r[0] for r in rseq], (k, gseq, rseq)
        np.testing.assert_allclose([g[1] for g in gseq], [r[1] for r in rseq], rtol=1e-6, atol=1e-6)
        n_multi += len(rseq) > 1
    assert n_multi >= 2  # the decoys really made trees


def test_permutation_invariance(oracle_lib, det_dense):
    """Shuffling measurements within each module and the order of seeds does
    not change any found track (rank keys are total orders)."""
    ev = make_event(det_dense, 5, mu=10)
    inp = oracle_lib.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev)
    ref = oracle_lib.ckf_find(inp, n_threads=4)
    rng = np.random.default_rng(0)
    perm = np.arange(ev.n_meas)
    for s in range(ev.n_surfaces):
        a, b = ev.offsets[s], ev.offsets[s + 1]
        perm[a:b] = a + rng.permutation(b - a)
    ev2 = make_event(det_dense, 5, mu=10)
    ev2.loc, ev2.var = ev.loc[perm], ev.var[perm]
    sp = rng.permutation(ev.n_seeds)
    ev2.seed_event, ev2.seed_surface = ev.seed_event[sp], ev.seed_surface[sp]
    ev2.seed_params, ev2.seed_cov = ev.seed_params[sp], ev.seed_cov[sp]
    inp2 = oracle_lib.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev2)
    got = oracle_lib.ckf_find(inp2, n_threads=4)
    assert got["n_tracks"] == ref["n_tracks"]
    by_seed = {sp[got["seed"][t]]: t for t in range(got["n_tracks"])}
    for t in range(ref["n_tracks"]):
        u = by_seed[ref["seed"][t]]
        a = ref["meas"][ref["offsets"][t]:ref["offsets"][t + 1]]
        b = perm[got["meas"][got["offsets"][u]:got["offsets"][u + 1]]]
        assert list(a) == list(b)
        assert np.array_equal(ref["params"][t], got["params"][u])
        assert np.array_equal(ref["cov"][t], got["cov"][u])
