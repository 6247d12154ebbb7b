"""The learned next-module proposal on the GPU, through the C ABI, against
the FP64 oracle (neighbour table, network forward and gradient, Adam, pair
capture) and against the plain GPU search (the proposal changes nothing
where its listing equals the geometric one)."""
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


def _rand_params(seed):
    from oracle import learned as OL
    rng = np.random.Generator(np.random.PCG64(seed))
    P = OL.unpack_params(OL.init_params(seed).astype(np.float64))
    for b in ("b1", "b2", "b3"):
        P[b][:] = rng.normal(0, 0.2, P[b].shape)
    return OL.pack_params(P).astype(np.float32)


def test_neighbour_table_matches_oracle(ckf, det_dense):
    """The library's table (built on the host in FP64 from the FP32
    geometry) equals the oracle's: next layers and cell regions exactly,
    anchors and pitches to FP32 rounding."""
    from oracle import learned as OL
    _say("# neighbour table, barrel+endcap")
    g = det_dense.as_arrays()
    geo = ckf.Geometry(g)
    nxt, anc, reg = ckf.neighbours(geo)
    rng = np.random.Generator(np.random.PCG64(21))
    mods = np.sort(rng.choice(g["center"].shape[0], 600, replace=False))
    onxt, oreg, oanc = OL.neighbour_table(g, modules=mods)
    np.testing.assert_array_equal(nxt[mods], onxt)
    np.testing.assert_array_equal(reg[mods], oreg)
    used = onxt >= 0
    A = oanc[..., :3]
    phi = np.arctan2(A[..., 1], A[..., 0])
    w = np.where(g["layer_type"][np.maximum(onxt, 0)] == 0, A[..., 2], np.hypot(A[..., 0], A[..., 1]))
    want = np.stack([phi, w, oanc[..., 3], oanc[..., 4]], -1)
    np.testing.assert_allclose(anc[mods][used], want[used], rtol=1e-6, atol=1e-4)


def test_mlp_forward_matches_oracle(ckf):
    import torch
    from oracle import learned as OL
    _say("# network forward")
    rng = np.random.Generator(np.random.PCG64(4))
    for n in (1, 64, 203):
        params = _rand_params(n)
        x = rng.normal(0, 1, (n, 7)).astype(np.float32)
        model = ckf.Model(torch.as_tensor(params, device="cuda"))
        z = ckf.mlp_forward(model, torch.as_tensor(x, device="cuda")).cpu().numpy().astype(np.float64)
        zb = OL.forward(params, x, bf16=True)
        z64 = OL.forward(params, x)
        scale = max(1.0, np.abs(z64).max())
        assert np.abs(z - zb).max() <= 1e-3 * scale, np.abs(z - zb).max()
        assert np.abs(z - z64).max() <= 1e-2 * scale, np.abs(z - z64).max()


def test_mlp_grad_matches_oracle(ckf):
    import torch
    from oracle import learned as OL
    _say("# network gradient")
    rng = np.random.Generator(np.random.PCG64(5))
    for n in (37, 300):
        params = _rand_params(100 + n)
        x = rng.normal(0, 1, (n, 7)).astype(np.float32)
        lab = rng.integers(0, 32, n).astype(np.int32)
        dev = lambda a: torch.as_tensor(a, device="cuda")
        g, loss = ckf.mlp_grad(dev(params), dev(x), dev(lab))
        g = g.cpu().numpy().astype(np.float64)
        ol, og = OL.loss_and_grad(params.astype(np.float64), x.astype(np.float64), lab)
        cos = float(g @ og / (np.linalg.norm(g) * np.linalg.norm(og)))
        _say(f"#   n={n}: cosine to the FP64 gradient {cos:.6f}, loss {float(loss.item()):.5f} vs {ol:.5f}")
        assert cos >= 0.999
        assert abs(float(loss.item()) - ol) <= 1e-2 * ol
        # block by block against the oracle rounding to bf16 where the kernels do
        _, ob = OL.loss_and_grad(params.astype(np.float64), x.astype(np.float64), lab, bf16=True)
        G, B = OL.unpack_params(g), OL.unpack_params(ob)
        for k in G:
            rel = float(np.linalg.norm(G[k] - B[k]) / max(np.linalg.norm(B[k]), 1e-30))
            _say(f"#     {k}: relative error to the bf16-rounded oracle {rel:.2e}")
            assert rel <= 2e-3, k
        # a row-index array selects the same rows as the gathered copy, bitwise
        perm = rng.permutation(n).astype(np.int32)
        g2, _ = ckf.mlp_grad(dev(params), dev(x), dev(lab), rows=dev(perm))
        g3, _ = ckf.mlp_grad(dev(params), dev(x[perm]), dev(lab[perm]))
        assert torch.equal(g2, g3)


def test_mlp_adam_matches_oracle(ckf):
    import torch
    from oracle import learned as OL
    _say("# adam")
    rng = np.random.Generator(np.random.PCG64(6))
    p = rng.normal(0, 1, 6752).astype(np.float32)
    m = rng.normal(0, 1e-3, 6752).astype(np.float32)
    v = rng.uniform(0, 1e-5, 6752).astype(np.float32)
    g = rng.normal(0, 1e-2, 6752).astype(np.float32)
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    P, M, V, G = dev(p), dev(m), dev(v), dev(g)
    ckf.mlp_adam(P, M, V, G, 7, lr=1e-3)
    # the hyper-parameters cross the interface as FP32: the oracle takes the same values
    f32 = lambda a: float(np.float32(a))
    op, om, ov = OL.adam_step(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                              g.astype(np.float64), 7, lr=f32(1e-3), beta1=f32(0.9), beta2=f32(0.999),
                              eps=f32(1e-8))
    np.testing.assert_allclose(M.cpu().numpy(), om, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(V.cpu().numpy(), ov, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(P.cpu().numpy(), op, rtol=1e-6, atol=1e-6)


def test_capture_pairs_matches_oracle(ckf, det_barrel):
    """The GPU capture kernel on the oracle's own tracks (uploaded) gives the
    oracle's pairs: the same pairs and labels (a label may move by one cell
    only where the crossing sits within 1e-4 of a cell edge, the FP32 and
    FP64 helix then rounding differently), inputs to FP32 rounding."""
    import torch
    import oracle
    from oracle import learned as OL
    _say("# pair capture, tiny event")
    g = det_barrel.as_arrays()
    ev = make_event(det_barrel, 1, kind="tiny")
    inp = oracle.Inputs(g, (0, 0, 2.0), ev)
    r = oracle.ckf_find(inp, material_on=0)
    geo = ckf.Geometry(g)
    fld = ckf.UniformField(0, 0, 2.0)
    mods = np.unique(r["meas_surface"])
    n_mod = g["center"].shape[0]
    sn, sr, sa = OL.neighbour_table(g, modules=mods)
    onxt = np.full((n_mod, 3), -1, np.int32)
    oreg = np.full((n_mod, 3, 192), -1, np.int32)
    oanc = np.zeros((n_mod, 3, 5))
    onxt[mods], oreg[mods], oanc[mods] = sn, sr, sa
    x_o, lab_o, trk_o, pos_o, drop_o = OL.capture_pairs(g, onxt, oreg, oanc, r["offsets"], r["meas_surface"],
                                                        r["meas_params"])
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    out = dict(n_tracks=dev(np.array([r["n_tracks"]], np.int32)), offsets=dev(r["offsets"].astype(np.int32)),
               meas_surface=dev(r["meas_surface"].astype(np.int32)), meas_params=dev(r["meas_params"]))
    x, lab, trk, n_pairs, dropped = ckf.capture_pairs(geo, fld, out, 4096)
    _say(f"#   pairs {n_pairs} (oracle {len(lab_o)}), dropped {dropped} (oracle {drop_o})")
    assert n_pairs == len(lab_o) and dropped == drop_o
    x, lab, trk = x.cpu().numpy(), lab.cpu().numpy(), trk.cpu().numpy()
    np.testing.assert_array_equal(trk, trk_o)
    edge = (np.abs(np.abs(x_o[:, 0]) - 0.5) < 1e-4) | (np.abs(np.abs(x_o[:, 1]) - 0.5) < 1e-4)
    same = lab == lab_o
    assert np.all(same | edge)
    np.testing.assert_allclose(x[same & ~edge], x_o[same & ~edge], rtol=0, atol=2e-5)
    # a short capacity keeps the first pairs and still counts all of them
    x2, lab2, _, n2, _ = ckf.capture_pairs(geo, fld, out, 17)
    assert n2 == n_pairs and np.array_equal(lab2.cpu().numpy(), lab[:17])


def test_capture_pairs_many_tracks_matches_oracle(ckf, det_dense):
    """600 truth trajectories of a dense event, given as found tracks (the
    seeded generator's crossings: surface, local position, direction, q/p),
    span three capture blocks: the GPU capture gives the oracle's pairs in
    the same track and measurement order, and a capacity cut inside the
    second block keeps exactly the first pairs."""
    import torch
    from oracle import learned as OL
    _say("# pair capture, 600 truth tracks")
    g = det_dense.as_arrays()
    ev = make_event(det_dense, 11, mu=12)
    tr = ev.truth
    _, first = np.unique(tr.particle, return_index=True)
    offsets = np.append(first, len(tr.particle)).astype(np.int32)
    d = tr.dir
    mp = np.stack([tr.loc[:, 0], tr.loc[:, 1], np.arctan2(d[:, 1], d[:, 0]), np.arccos(np.clip(d[:, 2], -1, 1)),
                   tr.qop], -1)
    ms = tr.surface.astype(np.int32)
    n_t = len(first)
    assert n_t > 512
    mods = np.unique(ms)
    n_mod = g["center"].shape[0]
    sn, sr, sa = OL.neighbour_table(g, modules=mods)
    onxt = np.full((n_mod, 3), -1, np.int32)
    oreg = np.full((n_mod, 3, 192), -1, np.int32)
    oanc = np.zeros((n_mod, 3, 5))
    onxt[mods], oreg[mods], oanc[mods] = sn, sr, sa
    x_o, lab_o, trk_o, _, drop_o = OL.capture_pairs(g, onxt, oreg, oanc, offsets, ms, mp)
    geo = ckf.Geometry(g)
    fld = ckf.UniformField(0, 0, 2.0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    out = dict(n_tracks=dev(np.array([n_t], np.int32)), offsets=dev(offsets), meas_surface=dev(ms),
               meas_params=dev(mp))
    x, lab, trk, n_pairs, dropped = ckf.capture_pairs(geo, fld, out, len(lab_o) + 10)
    _say(f"#   pairs {n_pairs} (oracle {len(lab_o)}), dropped {dropped} (oracle {drop_o})")
    assert n_pairs == len(lab_o) and dropped == drop_o
    x, lab, trk = x.cpu().numpy(), lab.cpu().numpy(), trk.cpu().numpy()
    np.testing.assert_array_equal(trk, trk_o)
    assert trk.max() >= 2 * 256  # pairs from the third block
    edge = (np.abs(np.abs(x_o[:, 0]) - 0.5) < 1e-4) | (np.abs(np.abs(x_o[:, 1]) - 0.5) < 1e-4)
    same = lab == lab_o
    assert np.all(same | edge) and same.mean() > 0.99
    np.testing.assert_allclose(x[same & ~edge], x_o[same & ~edge], rtol=0, atol=2e-5)
    cut = int(np.searchsorted(trk_o, 300)) + 3  # inside the second block's pairs
    x2, lab2, trk2, n2, _ = ckf.capture_pairs(geo, fld, out, cut)
    assert n2 == n_pairs and len(lab2) == cut
    np.testing.assert_array_equal(lab2.cpu().numpy(), lab[:cut])
    np.testing.assert_array_equal(trk2.cpu().numpy(), trk[:cut])


@pytest.fixture(scope="module")
def trained(ckf, det_dense):
    """A network trained on the GPU on pairs from the plain GPU search of
    two dense events (a small stand-in for the full training set)."""
    from paper_2505_22822_amd import learned
    _say("# training on two mu=200 events")
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    batches = [ckf.Batch.from_event(make_event(det_dense, 5000 + i, mu=200)) for i in range(2)]
    params, log, info = learned.train_from_batches(geo, fld, batches, epochs=8, batch=2048, seed=1)
    _say(f"#   pairs {info['pairs']} dropped {info['dropped']} loss {log.loss[0]:.3f} -> {log.loss[-1]:.3f} "
         f"val top1 {log.val_top1:.3f} top3 {log.val_top3:.3f} confident {log.val_confident:.3f} "
         f"(right {log.val_confident_right:.4f})")
    return geo, fld, params, log, info


def test_training_learns(trained):
    """Training on the GPU lowers the loss; the validation figures are
    reported (how well the network can learn depends on the table and the
    input encoding)."""
    geo, fld, params, log, info = trained
    assert info["pairs"] > 50000
    # (overlapping modules give rows with two labels, so the loss stays above their entropy)
    assert log.loss[-1] < 0.6 * log.loss[0]
    assert log.val_top3 >= 0.9


def test_learned_search_equals_plain_where_listing_agrees(ckf, det_dense, trained):
    """Instrumented learned run: every seed whose candidates never used a
    proposal listing different from the geometric one finds exactly the
    plain search's track; with an unreachable confidence threshold every
    navigation falls back and the whole output equals the plain one."""
    geo, fld, params, log, info = trained
    ev = make_event(det_dense, 6000, mu=200)
    b = ckf.Batch.from_event(ev)
    model = ckf.Model(params)
    plain = ckf.find(geo, fld, b)
    learned = ckf.find(geo, fld, b, model=model, seed_flags=True)
    cnt = learned["counters"]
    _say(f"# learned counters: navigations {cnt['navigations']} network rows {cnt['mlp_rows']} "
         f"proposals {cnt['proposals']} misses {cnt['proposal_misses']} listing tests {cnt['nav_modules']} "
         f"(plain {plain['counters']['nav_modules']})")
    assert cnt["mlp_rows"] > 0.5 * cnt["navigations"]
    assert cnt["proposals"] > 0.1 * cnt["mlp_rows"]  # a network trained briefly on two events
    flags = learned["seed_flags"]
    pb = {int(s): t for t, s in enumerate(plain["seed"])}
    lb = {int(s): t for t, s in enumerate(learned["seed"])}
    n_same = 0
    for s in range(b.n_seeds):
        if flags[s]:
            continue
        tp, tl = pb.get(s), lb.get(s)
        assert (tp is None) == (tl is None), s
        if tp is None:
            continue
        a = plain["meas"][plain["offsets"][tp]:plain["offsets"][tp + 1]]
        c = learned["meas"][learned["offsets"][tl]:learned["offsets"][tl + 1]]
        assert np.array_equal(a, c), s
        assert np.array_equal(plain["params"][tp], learned["params"][tl]), s
        n_same += 1
    _say(f"#   flagged seeds {int(flags.sum())} of {b.n_seeds}; unflagged tracks identical: {n_same}")
    assert flags.sum() < 0.5 * b.n_seeds
    never = ckf.find(geo, fld, b, cfg=ckf.config(learned_min_prob=2.0), model=model)
    assert never["counters"]["proposals"] == 0 and never["counters"]["mlp_rows"] > 0
    for k in ("offsets", "meas", "params", "cov"):
        assert np.array_equal(never[k], plain[k]), k
    # the uninstrumented learned kernels find the same tracks as the instrumented one
    for waves in (1, 2, 3):
        f = ckf.Finder(geo, fld, b, ckf.config(), ckf.launch(0, 0, 64, None, waves), counters=False, model=model)
        f.enqueue()
        r = f.result()
        for k in ("offsets", "meas", "params"):
            assert np.array_equal(r[k], learned[k]), (waves, k)


def test_trained_network_saves_listing_work(ckf, det_dense, trained):
    """What training gains over the search without it, on one mu = 200 event
    (instrumented runs): the untrained network (its initial weights) is never
    confident, so every navigation falls back to the geometric listing and
    the module tests equal the plain search's; the trained network is
    confident on a share of the rows and its proposals replace the grid
    listing there, so fewer modules are tested."""
    import torch
    from paper_2505_22822_amd import learned
    geo, fld, params, log, info = trained
    b = ckf.Batch.from_event(make_event(det_dense, 6001, mu=200))
    plain = ckf.find(geo, fld, b)
    fresh = ckf.find(geo, fld, b, model=ckf.Model(torch.as_tensor(learned.init_params(1), device="cuda")))
    tuned = ckf.find(geo, fld, b, model=ckf.Model(params))
    cp, cf, ct = plain["counters"], fresh["counters"], tuned["counters"]
    _say(f"# listing module tests: plain {cp['nav_modules']}, untrained {cf['nav_modules']} "
         f"({cf['proposals']} proposals of {cf['mlp_rows']} rows), trained {ct['nav_modules']} "
         f"({ct['proposals']} proposals of {ct['mlp_rows']} rows)")
    # (the initial weights' summed top-3 probability stays below 0.8 over the inputs' whole range)
    assert cf["proposals"] == 0 and cf["nav_modules"] == cp["nav_modules"]
    assert ct["proposals"] >= 0.1 * ct["mlp_rows"]
    # (seen: 13 % fewer, 806,568 against 927,099, with 27 % of the rows confident)
    assert ct["nav_modules"] < 0.95 * cp["nav_modules"]
