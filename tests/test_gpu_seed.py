"""Triplet seeding on the GPU (ckf_seed) against the oracle on the same
spacepoints: the same triplets in the same order and the same parameters on
the oracle's clusters of a mu = 20 event; sampled middle spacepoints of an
8 x mu = 200 batch of measurements; the chain cells -> clusters -> seeds ->
tracks on the GPU; edge cases.  The spacepoints both sides take are the
oracle's (its clusters, or its spacepoint definition applied to the
measurements), rounded to FP32 once."""
import sys

import numpy as np
import pytest

from synth import make_event
from synth.cells import cell_grid, make_cells

pytestmark = pytest.mark.gpu
LAYERS = [0, 1, 2, 3]   # the pixel barrel layers of the dense detector, outwards


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


def _clusters_on_device(det, cells, ckf):
    import torch
    geo = ckf.Geometry(det.as_arrays())
    _, pitch = cell_grid(det)
    cl = ckf.Clusterer(geo, ckf.CellBatch.from_cells(cells), torch.as_tensor(pitch, device="cuda"))
    cl.enqueue()
    r = cl.result()
    m = r["n_meas"]
    return geo, cl, r, m


def _upload(offsets, xyz, loc):
    import torch
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return t(offsets, torch.int32), t(xyz, torch.float32), t(loc, torch.float32)


def _measurement_spacepoints(det, ev):
    """Spacepoints of an event's (or batch's) measurements by the oracle's
    definition, rounded to FP32: (offsets, xyz, loc)."""
    from oracle import clustering as OC
    S = det.n_surfaces
    rows = np.repeat(np.arange(ev.n_events * S), np.diff(ev.offsets))
    xyz = OC.spacepoints(det.as_arrays(), rows % S, ev.loc).astype(np.float32)
    return np.asarray(ev.offsets, np.int32), xyz, np.asarray(ev.loc, np.float32)


def _layer_index(det, offsets, n_events):
    S = det.n_surfaces
    rows = np.repeat(np.arange(n_events * S), np.diff(offsets))
    layer = det.as_arrays()["layer"][rows % S]
    li = np.full(len(rows), -1)
    for k, L in enumerate(LAYERS):
        li[layer == L] = k
    return li, rows


def test_seed_matches_oracle(ckf, det_dense):
    """A mu = 20 event's clusters: the GPU's seeds are the oracle's, triplet
    by triplet in the same order, on the same modules, with parameters to
    1e-12 relative (FP64 on both sides); with the tops of every middle held
    on chip (default), with none (every bottom scans its window) and with a
    capacity that some middles exceed."""
    from oracle import clustering as OC, seeding as OS
    ev = make_event(det_dense, 6000, mu=20)
    cells = make_cells(det_dense, ev, 1)
    _, pitch = cell_grid(det_dense)
    oc = OC.cluster(cells, det_dense.as_arrays(), pitch)
    xyz, loc = oc["spacepoint"].astype(np.float32), oc["loc"].astype(np.float32)
    m = len(xyz)
    geo = ckf.Geometry(det_dense.as_arrays())
    d_off, d_xyz, d_loc = _upload(oc["offsets"], xyz, loc)
    li, rows = _layer_index(det_dense, oc["offsets"], 1)
    ref = OS.seeds(xyz.astype(np.float64), li, rows, loc.astype(np.float64), 2.0)
    try:
        for cap in (None, 0, 12):
            ckf.seed_top_cap(cap)
            sd, n = ckf.seed(geo, 1, d_off, d_xyz, d_loc, LAYERS, 2.0)
            _say(f"# seeding (top capacity {cap}): {m} spacepoints, {n} seeds (oracle {len(ref['middle'])})")
            sp = sd["spacepoints"].cpu().numpy()
            assert n == len(ref["middle"])
            np.testing.assert_array_equal(sp[:, 0], ref["bottom"])
            np.testing.assert_array_equal(sp[:, 1], ref["middle"])
            np.testing.assert_array_equal(sp[:, 2], ref["top"])
            np.testing.assert_array_equal(sd["surface"].cpu().numpy(), ref["surface"])
            assert np.all(sd["event"].cpu().numpy() == 0)
            p = sd["params"].cpu().numpy()
            np.testing.assert_allclose(p, ref["params"], rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(sd["cov"].cpu().numpy(), ref["cov"], rtol=1e-12, atol=0)
    finally:
        ckf.seed_top_cap(None)


@pytest.fixture(scope="module")
def batch200(ckf, det_dense):
    """Spacepoints of the measurements of 8 x mu = 200 events (the oracle's
    definition, FP32), on the host and on the device."""
    from synth import concat_events
    ev = concat_events([make_event(det_dense, 7100 + i, mu=200) for i in range(8)])
    off, xyz, loc = _measurement_spacepoints(det_dense, ev)
    return ckf.Geometry(det_dense.as_arrays()), (off, xyz, loc), _upload(off, xyz, loc)


def test_seed_batch_sampled_middles(ckf, det_dense, batch200):
    """8 x mu = 200 events in one call: for 400 sampled middle spacepoints
    the oracle, on that middle's event alone, keeps the same triplets."""
    from oracle import seeding as OS
    geo, (off, xyz32, _), dev = batch200
    m = len(xyz32)
    sd, n = ckf.seed(geo, 8, *dev, LAYERS, 2.0)
    sp = sd["spacepoints"].cpu().numpy()
    _say(f"# seeding batch: {m} spacepoints, {n} seeds")
    li, rows = _layer_index(det_dense, off, 8)
    S = det_dense.n_surfaces
    ev_of = rows // S
    xyz = xyz32.astype(np.float64)
    rng = np.random.default_rng(9)
    middles = rng.choice(np.nonzero((li == 1) | (li == 2))[0], 400, replace=False)
    for mid in middles:
        e = ev_of[mid]
        idx = np.nonzero(ev_of == e)[0]
        local = np.searchsorted(idx, mid)
        ref = OS.triplets(xyz[idx], li[idx], 2.0, middles=[local])
        got = sp[sp[:, 1] == mid]
        assert [(idx[b], idx[t]) for _, b, t, _ in ref] == [(int(a), int(c)) for a, _, c in got], mid


def test_seed_top_capacity_batch(ckf, batch200):
    """8 x mu = 200 events: the seeds are the same, bit for bit, whether the
    middles' tops are held on chip, never (every bottom scans its window),
    or up to a capacity that part of the middles exceed, and with or without
    the work counters.  The counters agree where the paths do the same work:
    every bottom is tested once per middle, and the same (B, M, T) triples
    reach the triplet test, on every path."""
    import torch
    geo, _, dev = batch200
    out, work = [], []
    try:
        for cap in (None, 0, 160):
            ckf.seed_top_cap(cap)
            w = torch.zeros(4, dtype=torch.int64, device="cuda")
            sd, n = ckf.seed(geo, 8, *dev, LAYERS, 2.0, counters=w)
            out.append((n, {k: v.cpu().numpy() for k, v in sd.items()}))
            work.append([int(x) for x in w.cpu()])
            _say(f"# seeding batch (top capacity {cap}): {n} seeds; work (MT, BM, cot, triplets) {work[-1]}")
        sd, n = ckf.seed(geo, 8, *dev, LAYERS, 2.0)  # (the last capacity, no counters)
        out.append((n, {k: v.cpu().numpy() for k, v in sd.items()}))
    finally:
        ckf.seed_top_cap(None)
    n0, ref = out[0]
    assert n0 > 100000
    for n, got in out[1:]:
        assert n == n0
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    for w in work:
        assert min(w) > 0 and w[2] >= w[3]
    assert all(w[1] == work[0][1] and w[3] == work[0][3] for w in work)


def test_chain_cells_to_tracks(ckf, det_dense):
    """cells -> clusters -> seeds -> tracks, all on the GPU, for a mu = 50
    event: most central particles (|eta| < 1.2, pT > 0.6 GeV, |z_vertex|
    < 150 mm) end with a track made mostly of their own clusters."""
    import torch
    ev = make_event(det_dense, 6200, mu=50)
    cells = make_cells(det_dense, ev, 4)
    geo, cl, r, m = _clusters_on_device(det_dense, cells, ckf)
    sd, n = ckf.seed(geo, 1, cl.offsets, cl.spacepoints[:m], cl.loc[:m], LAYERS, 2.0)
    cc = r["cell_cluster"]
    o = np.lexsort((-cells.q, cc))
    first = o[np.r_[True, cc[o][1:] != cc[o][:-1]]]
    cl_part = np.full(m, -1, np.int64)
    cl_part[cc[first]] = cells.particle[first]
    b = ckf.Batch(1, ev.n_surfaces, cl.offsets, cl.loc[:m].contiguous(), cl.var[:m].contiguous(),
                  sd["event"].contiguous(), sd["surface"].contiguous(), sd["params"].contiguous(),
                  sd["cov"].contiguous())
    res = ckf.find(geo, ckf.UniformField(0, 0, 2.0), b)
    found = set()
    for k in range(res["n_tracks"]):
        ids = res["meas"][res["offsets"][k]:res["offsets"][k + 1]]
        parts, cnt = np.unique(cl_part[ids], return_counts=True)
        j = int(np.argmax(cnt))
        if parts[j] >= 0 and cnt[j] > len(ids) / 2:
            found.add(int(parts[j]))
    cen = [p for p in range(len(ev.particle_pt))
           if abs(ev.particle_eta[p]) < 1.2 and ev.particle_pt[p] > 0.6 and abs(ev.particle_vtx[p, 2]) < 150]
    eff = np.mean([p in found for p in cen])
    _say(f"# chain: {m} clusters, {n} seeds, {res['n_tracks']} tracks, central particles found {eff:.4f}")
    assert len(cen) > 500 and eff > 0.95


def test_seed_edge_cases(ckf, det_dense):
    """No spacepoints; fewer than three or unknown seeding layers are
    rejected; a short capacity counts all seeds and writes the first."""
    import torch
    from paper_2505_22822_amd import CkfError
    geo = ckf.Geometry(det_dense.as_arrays())
    S = det_dense.n_surfaces
    off = torch.zeros(S + 1, dtype=torch.int32, device="cuda")
    z3 = torch.zeros((1, 3), dtype=torch.float32, device="cuda")
    z2 = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    sd, n = ckf.seed(geo, 1, off, z3[:0], z2[:0], LAYERS, 2.0)
    assert n == 0
    with pytest.raises(CkfError):
        ckf.seed(geo, 1, off, z3[:0], z2[:0], [0, 1], 2.0)
    with pytest.raises(CkfError):
        ckf.seed(geo, 1, off, z3[:0], z2[:0], [0, 1, 999], 2.0)
    ev = make_event(det_dense, 6000, mu=20)
    cells = make_cells(det_dense, ev, 1)
    geo, cl, r, m = _clusters_on_device(det_dense, cells, ckf)
    full, n_full = ckf.seed(geo, 1, cl.offsets, cl.spacepoints[:m], cl.loc[:m], LAYERS, 2.0)
    part, n_part = ckf.seed(geo, 1, cl.offsets, cl.spacepoints[:m], cl.loc[:m], LAYERS, 2.0, cap_seeds=100)
    assert n_part == n_full > 100 and part["params"].shape[0] == 100
    np.testing.assert_array_equal(part["spacepoints"].cpu().numpy(), full["spacepoints"][:100].cpu().numpy())


def test_seed_hand_placed_degenerate_cases(ckf, det_dense):
    """Hand-placed spacepoints on modules of the first three seeding layers,
    against the oracle case by case: points exactly on the x axis (zero
    circle determinant: no finite circle, no seed); a radial line at phi =
    0.3 (collinear up to rounding: a huge radius and d0 ~ 0, a seed); a
    curved helix of 2 GeV (a seed with the right charge sign); the middle
    moved 3 mm sideways (d0 cut fails); an azimuth step of 0.15 rad (no
    seed)."""
    import math
    import torch
    from oracle import seeding as OS
    g = det_dense.as_arrays()
    S = det_dense.n_surfaces
    mods = np.array([int(np.nonzero(g["layer"] == L)[0][0]) for L in LAYERS[:3]])  # one module per layer
    order = np.argsort(mods)  # spacepoints come in row (module id) order
    geo = ckf.Geometry(g)

    def run(xyz):
        off = np.zeros(S + 1, np.int32)
        for s in mods:
            off[s + 1:] += 1
        xyz32 = np.asarray(xyz, np.float32)[order]
        li = np.array([0, 1, 2])[order]
        loc = np.zeros((3, 2), np.float32)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
        sd, n = ckf.seed(geo, 1, t(off, torch.int32), t(xyz32, torch.float32), t(loc, torch.float32), LAYERS, 2.0)
        ref = OS.triplets(xyz32.astype(np.float64), li, 2.0)
        got = [tuple(int(v) for v in r) for r in sd["spacepoints"].cpu().numpy()]
        assert [(b, m, t_) for m, b, t_, _ in ref] == got
        return n, sd

    pt = lambda r, z, phi: [r * math.cos(phi), r * math.sin(phi), z]
    n, _ = run([[30.0, 0.0, 3.0], [70.0, 0.0, 7.0], [120.0, 0.0, 12.0]])
    assert n == 0  # exactly collinear
    n, _ = run([pt(30, 3, 0.3), pt(70, 7, 0.3), pt(120, 12, 0.3)])
    assert n == 1
    R = 2.0 / (OS.KAPPA * 2.0)  # a 2 GeV helix from the origin, turning clockwise (positive charge)
    arc = lambda r: [R * math.sin(2 * math.asin(r / (2 * R))) * 1.0, -R * (1 - math.cos(2 * math.asin(r / (2 * R)))), 0.1 * r]
    n, sd = run([arc(30), arc(70), arc(120)])
    assert n == 1 and sd["params"][0, 4].item() > 0
    side = [pt(30, 3, 0.3), pt(70, 7, 0.3), pt(120, 12, 0.3)]
    side[1][0] += -3.0 * math.sin(0.3)
    side[1][1] += 3.0 * math.cos(0.3)
    n, _ = run(side)
    assert n == 0
    n, _ = run([pt(30, 3, 0.3), pt(70, 7, 0.45), pt(120, 12, 0.6)])
    assert n == 0
