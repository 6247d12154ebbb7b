"""Pins of the oracle's learned search (no GPU).

The C++ track finder applies the learned next-module proposal inside the
search (the proposal replaces only the module lookup of the navigation,
paper section 2, and keeps that lookup as its fallback).  Its pieces are
pinned against the Python oracle's definitions, which are themselves pinned
by closed forms (tests/test_oracle_learned.py): the network pass against
``oracle.learned.forward`` in both precisions, and the window, input and
top-k of a proposal against ``crossing_window``, ``features_at`` and
``top3``.  The search as a whole reduces to the plain search where it must:
with an unreachable threshold, bit for bit; and for every seed none of
whose used proposals listed differently from the geometric lookup."""
import numpy as np
import pytest

import oracle
from oracle import learned as OL
from synth import make_event


def _rand_params(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = OL.unpack_params(OL.init_params(seed).astype(np.float64))
    for b in ("b1", "b2", "b3"):
        P[b][:] = rng.normal(0, 0.2, P[b].shape)
    return OL.pack_params(P).astype(np.float32)


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_equals_python_oracle(oracle_lib, bf16):
    rng = np.random.Generator(np.random.PCG64(31))
    for n in (1, 50):
        params = _rand_params(n)
        x = rng.normal(0, 1, (n, 7))
        got = oracle.mlp_forward(params, x, bf16=bf16)
        want = OL.forward(params, x, bf16=bf16)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def _crossings(det, n_tracks=300):
    """(module, next layer, crossing point, direction, q/p) at the layer
    changes of the oracle's tracks on a small event."""
    g = det.as_arrays()
    ev = make_event(det, 71, mu=20)
    r = oracle.ckf_find(oracle.Inputs(g, (0, 0, 2.0), ev))
    layer = np.asarray(g["layer"])
    out = []
    for t in range(min(n_tracks, r["n_tracks"])):
        for i in range(r["offsets"][t], r["offsets"][t + 1] - 1):
            m, m2 = int(r["meas_surface"][i]), int(r["meas_surface"][i + 1])
            L2 = int(layer[m2])
            if L2 == layer[m]:
                continue
            cr = OL.state_crossing(g, m, r["meas_params"][i], L2)
            if cr is not None:
                out.append((m, L2, cr[0], cr[1], float(r["meas_params"][i][4])))
    return out


def test_proposal_pieces_equal_python_oracle(oracle_lib, det_dense, dense_table, golden_model):
    """Window cell, network input, summed top-3 probability, the three most
    probable outputs and their modules of the C++ proposal equal the Python
    oracle's definitions at the layer changes of found tracks."""
    g = det_dense.as_arrays()
    nxt, reg, anc = dense_table
    lrn = oracle.LearnedInputs(dense_table, golden_model, min_prob=0.95)
    inp = oracle.Inputs(g, (0, 0, 2.0))
    n_checked = n_used = 0
    for m, L2, X, T, qop in _crossings(det_dense):
        got = oracle.learned_propose(inp, lrn, m, L2, X, T, qop)
        slots = np.nonzero(nxt[m] == L2)[0]
        if len(slots) == 0:
            assert got is None
            continue
        s = slots[0]
        iu, iv, fu, fv = OL.crossing_window(g, L2, X, anc[m, s])
        assert got is not None
        assert (got["cell"][0], got["cell"][1]) == (iu, iv)
        want_x = OL.features_at(g, L2, X, T, qop, anc[m, s])
        np.testing.assert_allclose(got["features"], want_x, rtol=0, atol=1e-12)
        z = OL.forward(golden_model, want_x[None, :], bf16=True)
        idx, mass = OL.top3(z)
        assert abs(got["conf"] - mass[0]) < 1e-12
        assert list(got["classes"]) == list(idx[0])
        wm = OL.window_modules(g, L2, X, anc[m, s], reg[m, s])
        assert list(got["modules"]) == [int(wm[c]) for c in idx[0]]
        assert got["used"] == (mass[0] >= 0.95)
        n_checked += 1
        n_used += got["used"]
    assert n_checked > 500 and n_used > 0.1 * n_checked, (n_checked, n_used)


def test_unreachable_threshold_is_the_plain_search(oracle_lib, det_dense, dense_table, golden_model):
    """With a threshold above 1 the network runs but is never used: the
    tracks are bitwise the plain search's."""
    ev = make_event(det_dense, 72, mu=30)
    inp = oracle.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev)
    plain = oracle.ckf_find(inp)
    never = oracle.ckf_find(inp, learned=oracle.LearnedInputs(dense_table, golden_model, min_prob=2.0))
    assert never["stats"]["mlp_rows"] > 0.5 * never["stats"]["navigations"]
    assert never["stats"]["proposals"] == 0 and not never["differs"].any()
    for k in ("offsets", "meas", "params", "cov", "chi2", "seed"):
        assert np.array_equal(never[k], plain[k]), k
    assert never["stats"]["nav_modules"] == plain["stats"]["nav_modules"]


def test_learned_search_equals_plain_where_listing_agrees(oracle_lib, det_dense, dense_table, golden_model):
    """The proposal changes only which modules are listed.  Seeds none of
    whose used proposals listed differently from the geometric lookup find
    exactly the plain search's tracks; the proposals replace a share of the
    geometric lookups, and some listings differ."""
    ev = make_event(det_dense, 73, mu=60)
    inp = oracle.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev)
    plain = oracle.ckf_find(inp)
    lrn = oracle.ckf_find(inp, learned=oracle.LearnedInputs(dense_table, golden_model, min_prob=0.95))
    st = lrn["stats"]
    print(f"rows {st['mlp_rows']} of {st['navigations']} navigations, proposals {st['proposals']}, "
          f"differing listings {st['proposal_misses']}, seeds differing {int(lrn['differs'].sum())} "
          f"of {ev.n_seeds}; listing tests {st['nav_modules']} (plain {plain['stats']['nav_modules']})")
    assert st["proposals"] > 0.1 * st["mlp_rows"]
    assert 0 < lrn["differs"].sum() < 0.3 * ev.n_seeds
    assert st["nav_modules"] < plain["stats"]["nav_modules"]
    pb = {int(s): t for t, s in enumerate(plain["seed"])}
    lb = {int(s): t for t, s in enumerate(lrn["seed"])}
    n_same = 0
    for s in range(ev.n_seeds):
        if lrn["differs"][s]:
            continue
        tp, tl = pb.get(s), lb.get(s)
        assert (tp is None) == (tl is None), s
        if tp is None:
            continue
        a = plain["meas"][plain["offsets"][tp]:plain["offsets"][tp + 1]]
        c = lrn["meas"][lrn["offsets"][tl]:lrn["offsets"][tl + 1]]
        assert np.array_equal(a, c), s
        assert np.array_equal(plain["params"][tp], lrn["params"][tl]), s
        n_same += 1
    assert n_same > 0.5 * plain["n_tracks"]
