"""Greedy ambiguity resolution on the GPU (ckf_resolve) against the oracle's
sequential greedy: the same kept set, bit for bit, on the oracle's tracks of a
mu = 100 event and on random track sets with heavy sharing and deliberate key
ties; properties on the GPU's own search at mu = 200; edge cases."""
import ctypes as C
import sys

import numpy as np
import pytest

from synth import make_event

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ckf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22822_amd as ckf
    return ckf


def _dev_tracks(off, meas, chi2, ndf):
    import torch
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return dict(n_tracks=t(np.array([len(off) - 1]), torch.int32), offsets=t(off, torch.int32),
                meas=t(meas if len(meas) else np.zeros(1), torch.int32), chi2=t(chi2, torch.float64),
                ndf=t(ndf, torch.int32))


def _random_set(rng, n_t, n_m, span):
    """n_t tracks of 6-12 measurements drawn from n_m ids in local
    neighbourhoods of `span` ids (heavy sharing, long chains); chi2 with few
    distinct values, so many keys tie."""
    tracks = []
    for t in range(n_t):
        n = int(rng.integers(6, 13))
        c = int(rng.integers(0, n_m - span))
        tracks.append(np.sort(rng.choice(np.arange(c, c + span), n, replace=False)))
    off = np.zeros(n_t + 1, np.int32)
    off[1:] = np.cumsum([len(t) for t in tracks])
    meas = np.concatenate(tracks).astype(np.int32)
    chi2 = rng.integers(1, 6, n_t).astype(np.float64) * 2.5   # few distinct values: many ties
    ndf = np.array([2 * len(t) - 5 for t in tracks], np.int32)
    return off, meas, chi2, ndf, n_m


def test_resolve_matches_oracle_on_oracle_tracks(ckf, det_dense):
    import oracle
    from oracle import ambiguity as OA
    ev = make_event(det_dense, 41, mu=100)
    r = oracle.ckf_find(oracle.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev), n_threads=0)
    keep_o, order = OA.resolve(r["offsets"], r["meas"], r["chi2"], r["ndf"])
    keep, rounds = ckf.resolve(_dev_tracks(r["offsets"], r["meas"], r["chi2"], r["ndf"]), ev.n_meas)
    keep = keep.cpu().numpy()
    _say(f"# resolve: {r['n_tracks']} tracks, oracle removes {len(order)}, GPU rounds {rounds}")
    np.testing.assert_array_equal(keep == 1, keep_o)
    assert np.all(keep >= 0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_resolve_matches_oracle_on_random_sets(ckf, seed):
    """2,000 tracks of 6-12 measurements drawn from 3,000 ids in local
    neighbourhoods (heavy sharing, long chains), chi2/ndf with many exact
    ties and equal share fractions: the parallel rounds keep exactly the
    sequential greedy's set, for max_shared 0, 1 and 2."""
    from oracle import ambiguity as OA
    rng = np.random.default_rng(seed)
    off, meas, chi2, ndf, n_m = _random_set(rng, 2000, 3000, 40)
    for ms in (0, 1, 2):
        keep_o, order = OA.resolve(off, meas, chi2, ndf, max_shared=ms)
        keep, rounds = ckf.resolve(_dev_tracks(off, meas, chi2, ndf), n_m, max_shared=ms)
        _say(f"# random set {seed}, max_shared {ms}: oracle removes {len(order)}, GPU rounds {rounds}")
        np.testing.assert_array_equal(keep.cpu().numpy() == 1, keep_o)


def test_resolve_gpu_search_properties(ckf, det_dense):
    """The GPU's own search on a mu = 200 event: after resolution no kept
    track shares more than one measurement with the other kept tracks, and
    only a small fraction of the tracks goes."""
    ev = make_event(det_dense, 7, mu=200)
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    finder = ckf.Finder(geo, fld, ckf.Batch.from_event(ev), ckf.config(), counters=False)
    finder.enqueue()
    r = finder.result()
    keep, rounds = ckf.resolve(finder.out, ev.n_meas)
    keep = keep.cpu().numpy()[:r["n_tracks"]]
    off, meas = r["offsets"], r["meas"]
    use = np.bincount(meas[np.repeat(keep == 1, np.diff(off))], minlength=ev.n_meas)
    worst = max(int(np.sum(use[meas[off[t]:off[t + 1]]] > 1)) for t in np.nonzero(keep == 1)[0])
    _say(f"# resolve of the GPU search: {r['n_tracks']} tracks, removed {int(np.sum(keep == 0))}, rounds {rounds}")
    assert worst <= 1
    assert 0 < np.sum(keep == 0) < 0.02 * r["n_tracks"] and np.all(keep >= 0)


def test_resolve_edge_cases(ckf):
    """No tracks; a track with an id out of range and one with offsets past
    the capacity take no part (-1); a short workspace and a negative
    max_shared are rejected."""
    import torch
    from paper_2505_22822_amd import _abi
    t0 = _dev_tracks(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0, np.int32))
    keep, rounds = ckf.resolve(t0, 10)
    assert rounds == 0
    off = np.array([0, 6, 12, 40], np.int32)
    meas = np.array([0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 4, 99], np.int32)
    t1 = _dev_tracks(off, meas, np.ones(3), np.full(3, 7, np.int32))
    keep, _ = ckf.resolve(t1, 50)
    assert list(keep.cpu().numpy()) == [1, -1, -1]
    lib = _abi.load()
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    k = torch.zeros(3, dtype=torch.int32, device="cuda")
    args = [t1["n_tracks"].data_ptr(), 3, 12, t1["offsets"].data_ptr(), t1["meas"].data_ptr(), 50,
            t1["chi2"].data_ptr(), t1["ndf"].data_ptr()]
    assert lib.ckf_resolve(*args, 1, 8, ws.data_ptr(), 64, k.data_ptr(), None, None) == 3
    assert lib.ckf_resolve(*args, -1, 8, ws.data_ptr(), 64, k.data_ptr(), None, None) == 1
    assert lib.ckf_resolve(*args, 1, 0, ws.data_ptr(), 64, k.data_ptr(), None, None) == 1


def test_resolve_round_bound_and_graph_capture(ckf):
    """The rounds run on the device: a bound too small for a heavily shared
    set reports converged = 0 and a prefix of the greedy (its removals are
    among the greedy's); and the call, captured in a graph, replayed three
    times with eager work between, gives the eager result every time."""
    import torch
    import oracle.ambiguity as OA
    rng = np.random.default_rng(11)
    off, meas, chi2, ndf, n_m = _random_set(rng, 400, 900, 20)
    t = _dev_tracks(off, meas, chi2, ndf)
    keep_o, _ = OA.resolve(off, meas, chi2, ndf)
    keep, rounds = ckf.resolve(t, n_m)
    assert np.array_equal(keep.cpu().numpy(), keep_o)
    _say(f"[resolve] heavily shared set: {rounds} rounds")
    assert rounds >= 2
    k1, info = ckf.resolve(t, n_m, max_rounds=1, sync=False)
    torch.cuda.synchronize()
    assert list(info.cpu().numpy()) == [1, 0]
    k1 = k1.cpu().numpy()
    assert np.all(keep_o[k1 == 0] == 0) and np.sum(k1 == 0) < np.sum(keep_o == 0)
    # graph capture of the whole call (the rounds are on the device)
    s = torch.cuda.Stream()
    nb = C.c_size_t(0)
    from paper_2505_22822_amd import _abi
    assert _abi.load().ckf_resolve_workspace_size(len(off) - 1, n_m, C.byref(nb)) == 0
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        ckf.resolve(t, n_m, stream=s, workspace=ws, info=info, sync=False)  # warm-up outside the graph
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        kg, _ = ckf.resolve(t, n_m, stream=s, workspace=ws, info=info, sync=False)
    for rep in range(3):
        kg.fill_(7)
        info.zero_()
        _ = torch.ones(1000, device="cuda").sum()  # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(kg.cpu().numpy(), keep_o), rep
        assert list(info.cpu().numpy()) == [rounds, 1], rep
