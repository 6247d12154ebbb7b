"""Parity at the benchmark's full size: the 64 x mu = 200 batch the bench
times (events and cells of RNG seeds 6000...6063, made by the bench's own
generator), in the launch shapes the bench times, against the oracle on
sampled outputs it computes one by one:
* the plain search, in both launch shapes the autotuner picks between, on
  20,000 sampled seeds (tracks depend on their seed alone);
* the learned search in its timed launch shape and threshold: seeds whose
  proposals never differed from the geometric listing find the plain track;
* clustering of the batch's 9.8M cells, on 2,000 sampled (event, module)
  rows;
* seeding on the batch's 5.1M measurement spacepoints, on 300 sampled
  middle spacepoints;
* the fit (both smoothers) of the GPU's tracks, on 200 sampled tracks."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_EVENTS = 64
SEEDS = [6000 + i for i in range(N_EVENTS)]
PARAM_SCALE = np.array([10.0, 30.0, 1.0, 1.0, 0.0])
DIAG = [0, 5, 9, 12, 14]
LAYERS = [0, 1, 2, 3]


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


@pytest.fixture(scope="module")
def batch64(ckf):
    """The bench's batch: (events, concatenated event, concatenated cells).
    Generated in fresh worker processes (spawn), which touch no GPU."""
    import multiprocessing as mp
    import bench
    from synth import concat_events
    from synth.cells import concat_cells
    workers = min(16, len(os.sched_getaffinity(0)))
    _say(f"# generating the {N_EVENTS} x mu=200 batch with {workers} workers")
    with mp.get_context("spawn").Pool(workers) as pool:
        out = pool.map(bench._gen, [(s, 200.0, True) for s in SEEDS])
    evs = [e for e, _ in out]
    return evs, concat_events(evs), concat_cells([c for _, c in out])


@pytest.fixture(scope="module")
def geo_fld(ckf, det_dense):
    return ckf.Geometry(det_dense.as_arrays()), ckf.UniformField(0, 0, 2.0)


def _find(ckf, geo, fld, b, grid, spg, waves, model=None, cfg=None):
    f = ckf.Finder(geo, fld, b, cfg or ckf.config(), ckf.launch(grid=grid, seeds_per_group=spg, waves_per_simd=waves),
                   counters=False, model=model)
    f.enqueue()
    return f.result()


def test_search_full_batch_sampled_seeds(ckf, det_dense, batch64, geo_fld):
    """Plain search on the whole batch in the launch shape the bench times
    (grid 2048, 48 seeds per pop, 2 waves per SIMD): the other shapes the
    bench's autotuner chooses between give bitwise the same tracks; on
    20,000 sampled seeds the oracle finds the same patterns for >= 99.9 % of
    its tracks, with parameters within 1e-4 of their scale and covariance
    diagonals within 1e-4 relative."""
    import oracle
    evs, batch, _ = batch64
    geo, fld = geo_fld
    b = ckf.Batch.from_event(batch)
    _say(f"# full batch: {batch.n_seeds} seeds, {batch.n_meas} measurements")
    got = _find(ckf, geo, fld, b, 2048, 48, 2)
    for shape in ((4096, 48, 2), (2048, 32, 2), (3072, 48, 3), (6144, 32, 3)):
        _say(f"#   shape {shape}")
        other = _find(ckf, geo, fld, b, *shape)
        for k in ("offsets", "meas", "params", "cov", "chi2", "seed"):
            assert np.array_equal(other[k], got[k]), (shape, k)
    rng = np.random.default_rng(21)
    sel = np.sort(rng.choice(batch.n_seeds, 20000, replace=False))
    inp = oracle.Inputs(det_dense.as_arrays(), (0, 0, 2.0))
    inp.set_event(batch, seeds=sel)
    ref = oracle.ckf_find(inp, n_threads=0)
    gb = {int(s): t for t, s in enumerate(got["seed"])}
    same, mism, worst, cw = 0, [], np.zeros(5), 0.0
    ref_seeds = set()
    for t in range(ref["n_tracks"]):
        s = int(sel[ref["seed"][t]])
        ref_seeds.add(s)
        u = gb.get(s)
        a = ref["meas"][ref["offsets"][t]:ref["offsets"][t + 1]]
        if u is None or not np.array_equal(a, got["meas"][got["offsets"][u]:got["offsets"][u + 1]]):
            mism.append(s)
            continue
        same += 1
        pr, pg = ref["params"][t], got["params"][u]
        d = pg - pr
        d[2] = (d[2] + math.pi) % (2 * math.pi) - math.pi
        scale = np.maximum(np.abs(pr), PARAM_SCALE)
        scale[4] = abs(pr[4])
        worst = np.maximum(worst, np.abs(d) / scale)
        cw = max(cw, float(np.max(np.abs(got["cov"][u][DIAG] - ref["cov"][t][DIAG]) / ref["cov"][t][DIAG])))
    extra = [s for s in sel if int(s) in gb and int(s) not in ref_seeds]
    _say(f"#   sampled seeds: oracle {ref['n_tracks']} tracks, identical {same}, mismatched {len(mism)} "
         f"{mism[:5]}, extra {len(extra)}, worst param rel {worst}, worst cov diag {cw:.2e}")
    assert same >= 0.999 * ref["n_tracks"] and len(extra) <= 0.001 * ref["n_tracks"]
    assert np.all(worst < 1e-4) and cw < 1e-4
    assert got["status"][5] == 0


def test_learned_full_batch_equals_plain_where_listing_agrees(ckf, det_dense, batch64, geo_fld):
    """Learned search on the whole batch with a network trained briefly on
    two other events, at the threshold the bench chooses (0.97): the
    instrumented run flags every seed whose candidates used a proposal
    listing that differs from the geometric one; every other seed finds the
    plain track bit for bit; the uninstrumented kernel in the shapes the
    bench times (grid 2048 or 4096, 48 seeds per pop, 2 waves per SIMD)
    finds the instrumented run's tracks."""
    from paper_2505_22822_amd import learned
    from synth import make_event
    evs, batch, _ = batch64
    geo, fld = geo_fld
    batches = [ckf.Batch.from_event(make_event(det_dense, 5000 + i, mu=200)) for i in range(2)]
    params, log, info = learned.train_from_batches(geo, fld, batches, epochs=8, batch=2048, seed=1)
    model = ckf.Model(params)
    b = ckf.Batch.from_event(batch)
    cfg = ckf.config(learned_min_prob=0.97)
    plain = _find(ckf, geo, fld, b, 2048, 48, 2, cfg=cfg)
    inst = ckf.find(geo, fld, b, cfg=cfg, model=model, seed_flags=True)
    flags = inst["seed_flags"]
    _say(f"# learned full batch: proposals {inst['counters']['proposals']}, flagged seeds {int(flags.sum())} "
         f"of {b.n_seeds}")
    assert inst["counters"]["proposals"] > 0 and flags.sum() < 0.5 * b.n_seeds
    pb = {int(s): t for t, s in enumerate(plain["seed"])}
    lb = {int(s): t for t, s in enumerate(inst["seed"])}
    for s in np.nonzero(flags == 0)[0]:
        tp, tl = pb.get(int(s)), lb.get(int(s))
        assert (tp is None) == (tl is None), s
        if tp is None:
            continue
        assert np.array_equal(plain["meas"][plain["offsets"][tp]:plain["offsets"][tp + 1]],
                              inst["meas"][inst["offsets"][tl]:inst["offsets"][tl + 1]]), s
        assert np.array_equal(plain["params"][tp], inst["params"][tl]), s
    for grid in (2048, 4096):
        timed = _find(ckf, geo, fld, b, grid, 48, 2, model=model, cfg=cfg)
        for k in ("offsets", "meas", "params", "seed"):
            assert np.array_equal(timed[k], inst[k]), (grid, k)


def test_cluster_full_batch_sampled_rows(ckf, det_dense, batch64):
    """Clustering of the batch's cells in one call: on 2,000 sampled
    non-empty (event, module) rows the oracle gives the same clusters and
    centroids (within one FP32 rounding)."""
    import torch
    from oracle import clustering as OC
    from synth.cells import Cells, cell_grid
    _, _, cells = batch64
    geo = ckf.Geometry(det_dense.as_arrays())
    _, pitch = cell_grid(det_dense)
    cl = ckf.Clusterer(geo, ckf.CellBatch.from_cells(cells), torch.as_tensor(pitch, device="cuda"))
    cl.enqueue()
    got = cl.result()
    _say(f"# full batch clustering: {cells.n_cells} cells, {got['n_meas']} clusters")
    assert got["status"] == 0 and got["offsets"][-1] == got["n_meas"]
    rows = np.nonzero(np.diff(cells.offsets) > 0)[0]
    rng = np.random.default_rng(22)
    S = cells.n_surfaces
    g = det_dense.as_arrays()
    for r in rng.choice(rows, 2000, replace=False):
        a, b = cells.offsets[r], cells.offsets[r + 1]
        s = r % S
        # the row alone, on a one-module geometry of its module
        one = Cells(1, 1, np.array([0, b - a], np.int32), cells.c0[a:b], cells.c1[a:b], cells.q[a:b],
                    cells.particle[a:b])
        g1 = {k: g[k][s:s + 1] for k in ("half", "rot", "center")}
        ref = OC.cluster(one, g1, pitch[s:s + 1])
        m0, m1 = got["offsets"][r], got["offsets"][r + 1]
        assert m1 - m0 == len(ref["size"]), r
        np.testing.assert_array_equal(got["cell_cluster"][a:b] - m0, ref["label"])
        assert np.all(np.abs(got["loc"][m0:m1] - ref["loc"]) <= 4e-6), r


def test_seed_full_batch_sampled_middles(ckf, det_dense, batch64):
    """Seeding on the spacepoints of the batch's 5.1M measurements (the
    oracle's definition, FP32) in one call: for 300 sampled middle
    spacepoints the oracle, on that middle's event alone, keeps the same
    triplets in the same order."""
    import torch
    from oracle import clustering as OC, seeding as OS
    _, batch, _ = batch64
    S = det_dense.n_surfaces
    rows = np.repeat(np.arange(batch.n_events * S), np.diff(batch.offsets))
    xyz = OC.spacepoints(det_dense.as_arrays(), rows % S, batch.loc).astype(np.float32)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    geo = ckf.Geometry(det_dense.as_arrays())
    sd, n = ckf.seed(geo, batch.n_events, t(batch.offsets, torch.int32), t(xyz, torch.float32),
                     t(batch.loc, torch.float32), LAYERS, 2.0)
    sp = sd["spacepoints"].cpu().numpy()
    _say(f"# full batch seeding: {len(xyz)} spacepoints, {n} seeds")
    layer = det_dense.as_arrays()["layer"][rows % S]
    li = np.full(len(rows), -1)
    for k, L in enumerate(LAYERS):
        li[layer == L] = k
    ev_of = rows // S
    x64 = xyz.astype(np.float64)
    rng = np.random.default_rng(23)
    order = np.argsort(sp[:, 1], kind="stable")
    for mid in rng.choice(np.nonzero((li == 1) | (li == 2))[0], 300, replace=False):
        idx = np.nonzero(ev_of == ev_of[mid])[0]
        ref = OS.triplets(x64[idx], li[idx], 2.0, middles=[np.searchsorted(idx, mid)])
        lo, hi = np.searchsorted(sp[order, 1], mid), np.searchsorted(sp[order, 1], mid, side="right")
        got = sp[order[lo:hi]]
        assert [(idx[b], idx[tt]) for _, b, tt, _ in ref] == [(int(a), int(c)) for a, _, c in got], mid


@pytest.mark.parametrize("smoother", ["rts", "two_filter"])
def test_fit_full_batch_sampled_tracks(ckf, det_dense, batch64, geo_fld, smoother):
    """Fit of the GPU search's tracks on the whole batch in one call: on 200
    sampled tracks the oracle's fit of the same measurements from the same
    seeds gives the smoothed states at every measurement within 1e-4 of
    their scale, covariance diagonals within 1e-4 relative."""
    import oracle
    from oracle import fit as OF
    _, batch, _ = batch64
    geo, fld = geo_fld
    b = ckf.Batch.from_event(batch)
    finder = ckf.Finder(geo, fld, b, ckf.config(), counters=False, meas_states=True)
    finder.enqueue()
    r = finder.result()
    f = ckf.Fitter.from_finder(finder, smoother)
    f.enqueue()
    g = f.result()
    assert np.mean(g["ok"][:r["n_tracks"]] == 1) >= 0.999
    inp = oracle.Inputs(det_dense.as_arrays(), (0, 0, 2.0), batch)
    rng = np.random.default_rng(24)
    worst, cworst = np.zeros(5), 0.0
    for t in rng.choice(r["n_tracks"], 200, replace=False):
        a, e = int(r["offsets"][t]), int(r["offsets"][t + 1])
        op, oc, _, ook = OF.fit_tracks(inp, batch, np.array([0, e - a]), r["meas"][a:e], r["meas_surface"][a:e],
                                       r["seed"][t:t + 1], "rts" if smoother == "rts" else "two")
        assert ook[0] == 1 and g["ok"][t] == 1, t
        d = g["params"][a:e] - op
        d[:, 2] = (d[:, 2] + math.pi) % (2 * math.pi) - math.pi
        scale = np.concatenate([np.broadcast_to(PARAM_SCALE[:4], (e - a, 4)), np.abs(op[:, 4:5])], 1)
        worst = np.maximum(worst, (np.abs(d) / np.maximum(np.abs(op), scale)).max(0))
        cworst = max(cworst, float((np.abs(g["cov"][a:e][:, DIAG] - oc[:, DIAG]) / oc[:, DIAG]).max()))
    _say(f"# full batch fit ({smoother}): {r['n_tracks']} tracks, sampled worst param rel {worst}, "
         f"cov diag {cworst:.2e}")
    assert np.all(worst < 1e-4) and cworst < 1e-4
