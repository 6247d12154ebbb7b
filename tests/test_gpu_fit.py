"""The Kalman-filter fit with its smoothers on the GPU (ckf_fit) against the
FP64 oracle's fit of the same tracks (the oracle's own track finding, uploaded),
plus properties that hold at any size on the GPU's own track finding (the
fitted fraction, unit-width smoothed pulls against truth); and the edge
cases (no tracks, ids out of range, a short workspace)."""
import math
import sys

import numpy as np
import pytest

from synth import make_event

pytestmark = pytest.mark.gpu

SCALE = np.array([10.0, 30.0, 1.0, 1.0])  # parameter scales of the tolerance (q/p: its own size)
DIAG = [0, 5, 9, 12, 14]


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
def oracle_event(det_dense):
    """A mu = 30 event and the oracle's tracks on it."""
    import oracle
    ev = make_event(det_dense, 31, mu=30)
    inp = oracle.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev)
    r = oracle.ckf_find(inp, n_threads=0)
    _say(f"# fit: {ev.n_seeds} seeds, oracle found {r['n_tracks']} tracks")
    return ev, inp, r


def _tracks_on_device(r, dev="cuda"):
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)
    return dict(n_tracks=t(np.array([r["n_tracks"]], np.int32)), offsets=t(r["offsets"].astype(np.int32)),
                meas=t(r["meas"].astype(np.int32)), meas_surface=t(r["meas_surface"].astype(np.int32)),
                seed=t(r["seed"].astype(np.int32)))


@pytest.mark.parametrize("smoother", ["rts", "two_filter"])
def test_fit_matches_oracle(ckf, det_dense, oracle_event, smoother):
    """Smoothed parameters at every measurement of the oracle's tracks:
    |gpu - oracle| <= 1e-4 max(|oracle|, scale) (scale 10 mm, 30 mm, 1 rad,
    1 rad, |q/p|), covariance diagonal within 1e-4 relative; every track
    fitted on both sides.  The fit's chi2 sums the forward residuals at the
    predicted positions, which the FP32 legs place to ~1e-5 mm: with a
    15 um resolution that moves each term by about 2 r dr / sigma^2 ~ 1e-3,
    so the sums agree to 2e-2 absolute."""
    from oracle import fit as OF
    ev, inp, r = oracle_event
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    b = ckf.Batch.from_event(ev)
    f = ckf.Fitter(geo, fld, b, _tracks_on_device(r), ckf.config(), smoother)
    f.enqueue()
    g = f.result()
    assert g["n_tracks"] == r["n_tracks"] and np.all(g["ok"] == 1)
    n = min(300, r["n_tracks"])  # the oracle fits the first tracks (Python loop)
    m = int(r["offsets"][n])
    op, oc, ochi2, ook = OF.fit_tracks(inp, ev, r["offsets"][:n + 1], r["meas"][:m], r["meas_surface"][:m],
                                       r["seed"][:n], "rts" if smoother == "rts" else "two")
    assert np.all(ook == 1)
    gp, gc = g["params"][:m], g["cov"][:m]
    d = gp - op
    d[:, 2] = (d[:, 2] + math.pi) % (2 * math.pi) - math.pi
    scale = np.concatenate([np.broadcast_to(SCALE, (m, 4)), np.abs(op[:, 4:5])], 1)
    rel = np.abs(d) / np.maximum(np.abs(op), scale)
    crel = np.abs(gc[:, DIAG] - oc[:, DIAG]) / oc[:, DIAG]
    _say(f"#   {smoother}: {m} states, params worst {rel.max(0)}, cov diag worst {crel.max(0)}")
    assert np.all(rel < 1e-4)
    assert np.all(crel < 1e-4)
    np.testing.assert_allclose(g["chi2"][:n], ochi2, rtol=0, atol=2e-2)


def test_fit_of_gpu_tracks_properties(ckf, det_dense):
    """The GPU's own search on a mu = 200 event, fitted on the GPU: every
    track is fitted; for truth-pure central tracks the smoothed pulls at
    every measurement have zero mean and unit width (both smoothers)."""
    ev = make_event(det_dense, 7, mu=200)
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    b = ckf.Batch.from_event(ev)
    finder = ckf.Finder(geo, fld, b, ckf.config(), counters=False, meas_states=True)
    finder.enqueue()
    r = finder.result()
    _say(f"# fit of the GPU search: {r['n_tracks']} tracks")
    tr = ev.truth
    key = {}
    for i in range(len(tr.particle)):
        key[(int(tr.particle[i]), int(tr.surface[i]))] = i
    for smoother in ("rts", "two_filter"):
        f = ckf.Fitter.from_finder(finder, smoother)
        f.enqueue()
        g = f.result()
        assert np.mean(g["ok"] == 1) >= 0.999 and np.all(g["ok"] >= 0)
        P = []
        for t in range(r["n_tracks"]):
            a, e = r["offsets"][t], r["offsets"][t + 1]
            ids = r["meas"][a:e]
            part = ev.seed_particle[r["seed"][t]]
            if not np.all(ev.meas_particle[ids] == part):
                continue
            rows = [key.get((int(part), int(s))) for s in r["meas_surface"][a:e]]
            if any(x is None for x in rows):
                continue
            d = tr.dir[rows]
            if abs(d[0, 2]) > 0.6:
                continue
            truth = np.stack([tr.loc[rows, 0], tr.loc[rows, 1], np.arctan2(d[:, 1], d[:, 0]),
                              np.arccos(np.clip(d[:, 2], -1, 1)), tr.qop[rows]], -1)
            diff = g["params"][a:e] - truth
            diff[:, 2] = (diff[:, 2] + math.pi) % (2 * math.pi) - math.pi
            P.append(diff / np.sqrt(g["cov"][a:e][:, DIAG]))
        P = np.concatenate(P)
        _say(f"#   {smoother}: {len(P)} states, pull mean {P.mean(0).round(3)}, std {P.std(0).round(3)}")
        assert len(P) > 5000
        np.testing.assert_allclose(P.mean(0), 0.0, atol=0.08)
        np.testing.assert_allclose(P.std(0), 1.0, atol=0.1)


def test_fit_edge_cases(ckf, det_dense):
    """No tracks; a track with a measurement id out of range (ok -1, NaN
    outputs); offsets beyond the capacity (ok -1, outputs untouched); a
    track longer than the finder's 64 steps (ok -1, NaN outputs) beside an
    empty one (ok 1) and a normal one (fitted); tracks whose ranges overlap
    (ok -1, outputs untouched); a short workspace (CKF_ERR_CAPACITY); an
    unknown smoother."""
    import torch
    import ctypes as C
    from paper_2505_22822_amd import _abi
    ev = make_event(det_dense, 3, mu=2)
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    b = ckf.Batch.from_event(ev)
    dev = lambda a: torch.as_tensor(np.asarray(a), device="cuda")
    # no tracks
    t0 = dict(n_tracks=dev(np.array([0], np.int32)), offsets=dev(np.zeros(3, np.int32)),
              meas=dev(np.zeros(4, np.int32)), meas_surface=dev(np.zeros(4, np.int32)), seed=dev(np.zeros(2, np.int32)))
    f = ckf.Fitter(geo, fld, b, t0)
    f.enqueue()
    assert f.result()["n_tracks"] == 0
    # two tracks: the first has an id out of range, the second offsets beyond the capacity
    s = int(ev.seed_surface[0])
    t1 = dict(n_tracks=dev(np.array([2], np.int32)), offsets=dev(np.array([0, 2, 9], np.int32)),
              meas=dev(np.array([0, ev.n_meas + 5, 0, 0], np.int32)),
              meas_surface=dev(np.array([s, s, s, s], np.int32)), seed=dev(np.zeros(2, np.int32)))
    f = ckf.Fitter(geo, fld, b, t1)
    f.params.fill_(7.0)
    f.enqueue()
    g = f.result()
    assert list(g["ok"]) == [-1, -1]
    p = f.params.cpu().numpy()
    assert np.all(np.isnan(p[:2])) and np.all(p[2:] == 7.0)
    # 65 measurements on the seed's module; an empty track; one measurement;
    # 64 measurements (the longest fitted)
    t2 = dict(n_tracks=dev(np.array([4], np.int32)), offsets=dev(np.array([0, 65, 65, 66, 130], np.int32)),
              meas=dev(np.zeros(130, np.int32)), meas_surface=dev(np.full(130, s, np.int32)),
              seed=dev(np.zeros(4, np.int32)))
    f = ckf.Fitter(geo, fld, b, t2)
    f.enqueue()
    g = f.result()
    assert list(g["ok"]) == [-1, 1, 1, 1]
    p = f.params.cpu().numpy()
    assert np.all(np.isnan(p[:65])) and np.all(np.isfinite(p[65:130]))
    # offsets going back: the first and the third track share measurements,
    # 5 in all against a capacity of 3 (the second track's range is reversed)
    t3 = dict(n_tracks=dev(np.array([3], np.int32)), offsets=dev(np.array([0, 3, 1, 3], np.int32)),
              meas=dev(np.zeros(3, np.int32)), meas_surface=dev(np.full(3, s, np.int32)),
              seed=dev(np.zeros(3, np.int32)))
    f = ckf.Fitter(geo, fld, b, t3)
    f.params.fill_(7.0)
    f.enqueue()
    g = f.result()
    assert list(g["ok"]) == [-1, -1, -1] and np.all(f.params.cpu().numpy() == 7.0)
    lib = _abi.load()
    cfg = ckf.config()
    assert lib.ckf_fit(geo.handle, fld.handle, C.byref(f._meas), C.byref(f._seeds), C.byref(cfg),
                       f.tracks["n_tracks"].data_ptr(), 2, 4, f.tracks["offsets"].data_ptr(),
                       f.tracks["meas"].data_ptr(), f.tracks["meas_surface"].data_ptr(),
                       f.tracks["seed"].data_ptr(), 0, f.workspace.data_ptr(), 16, f.params.data_ptr(),
                       f.cov.data_ptr(), f.chi2.data_ptr(), f.ok.data_ptr(), None) == 3
    assert lib.ckf_fit(geo.handle, fld.handle, C.byref(f._meas), C.byref(f._seeds), C.byref(cfg),
                       f.tracks["n_tracks"].data_ptr(), 2, 4, f.tracks["offsets"].data_ptr(),
                       f.tracks["meas"].data_ptr(), f.tracks["meas_surface"].data_ptr(),
                       f.tracks["seed"].data_ptr(), 2, f.workspace.data_ptr(), f.workspace.numel(),
                       f.params.data_ptr(), f.cov.data_ptr(), f.chi2.data_ptr(), f.ok.data_ptr(), None) == 1


@pytest.mark.parametrize("smoother", ["rts", "two_filter"])
def test_fit_tracks_on_the_seed_module(ckf, det_dense, oracle_event, smoother):
    """Tracks the search does not make, fitted against the oracle: one
    measurement on the seed's own module (no leg; smoothed = filtered), and
    two measurements of the seed's module in a row (a second update with no
    leg between; the RTS step then rebuilds the prediction without a
    transport).  Same tolerances as the fit of the oracle's tracks."""
    import torch
    from oracle import fit as OF
    ev, inp, _ = oracle_event
    seeds = [s for s in range(ev.n_seeds)
             if ev.offsets[ev.seed_surface[s] + 1] - ev.offsets[ev.seed_surface[s]] >= 2][:40]
    assert len(seeds) >= 10
    off, meas, msurf, seed = [0], [], [], []
    for k, s in enumerate(seeds):
        sf = int(ev.seed_surface[s])
        a = int(ev.offsets[sf])
        ids = [a] if k % 2 == 0 else [a, a + 1]
        meas += ids
        msurf += [sf] * len(ids)
        seed.append(s)
        off.append(len(meas))
    off, meas, msurf, seed = (np.array(x, np.int32) for x in (off, meas, msurf, seed))
    dev = lambda x: torch.as_tensor(x, device="cuda")
    tr = dict(n_tracks=dev(np.array([len(seed)], np.int32)), offsets=dev(off), meas=dev(meas),
              meas_surface=dev(msurf), seed=dev(seed))
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    f = ckf.Fitter(geo, fld, ckf.Batch.from_event(ev), tr, ckf.config(), smoother)
    f.enqueue()
    g = f.result()
    op, oc, ochi2, ook = OF.fit_tracks(inp, ev, off, meas, msurf, seed, "rts" if smoother == "rts" else "two")
    assert np.all(ook == 1) and np.all(g["ok"] == 1)
    d = g["params"] - op
    d[:, 2] = (d[:, 2] + math.pi) % (2 * math.pi) - math.pi
    m = len(meas)
    scale = np.concatenate([np.broadcast_to(SCALE, (m, 4)), np.abs(op[:, 4:5])], 1)
    rel = np.abs(d) / np.maximum(np.abs(op), scale)
    crel = np.abs(g["cov"][:, DIAG] - oc[:, DIAG]) / oc[:, DIAG]
    _say(f"#   {smoother} on the seed module: {len(seed)} tracks, params worst {rel.max(0)}, cov worst {crel.max():.2e}")
    assert np.all(rel < 1e-4) and np.all(crel < 1e-4)
    np.testing.assert_allclose(g["chi2"], ochi2, rtol=0, atol=2e-2)
