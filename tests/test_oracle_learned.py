"""Pins of the oracle's learned-proposal pieces (no GPU): the network's
gradient against central finite differences and closed forms, Adam against
its closed form for a constant gradient, bf16 rounding against exact
values, the network wiring against a hand-built network, and the neighbour
table against truth trajectories and geometric invariants."""
import numpy as np
import pytest

from oracle import learned as OL


def _rand_problem(n=24, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = OL.init_params(seed).astype(np.float64)
    params[OL.N_PARAMS - 32:] = rng.normal(0, 0.1, 32)  # non-zero output biases
    P = OL.unpack_params(params)
    P["b1"][:] = rng.normal(0, 0.1, 64)
    P["b2"][:] = rng.normal(0, 0.1, 64)
    params = OL.pack_params(P)
    x = rng.normal(0, 1, (n, 7))
    labels = rng.integers(0, 32, n).astype(np.int32)
    return params, x, labels


def test_gradient_matches_central_differences():
    params, x, labels = _rand_problem()
    loss, g = OL.loss_and_grad(params, x, labels)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.concatenate([rng.choice(OL.N_PARAMS, 300, replace=False), np.arange(OL.N_PARAMS - 32, OL.N_PARAMS)])
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (OL.loss_and_grad(pp, x, labels)[0] - OL.loss_and_grad(pm, x, labels)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])
    assert np.isfinite(loss) and loss > 0


def test_output_layer_closed_form():
    """With W3 = 0 every row's logits are b3: the loss is logsumexp(b3) minus
    the mean of b3 at the labels, the b3 gradient is softmax(b3) minus the
    label frequencies, and nothing below the output layer gets a gradient."""
    params, x, labels = _rand_problem(n=40)
    P = OL.unpack_params(params)
    P["W3"][:] = 0.0
    beta = np.linspace(-1.0, 2.0, 32)
    P["b3"][:] = beta
    params = OL.pack_params(P)
    loss, g = OL.loss_and_grad(params, x, labels)
    e = np.exp(beta - beta.max())
    soft = e / e.sum()
    lse = beta.max() + np.log(e.sum())
    assert abs(loss - (lse - beta[labels].mean())) < 1e-12
    freq = np.bincount(labels, minlength=32) / len(labels)
    G = OL.unpack_params(g)
    np.testing.assert_allclose(G["b3"], soft - freq, atol=1e-14)
    for k in ("W1", "b1", "W2", "b2"):
        assert np.all(G[k] == 0.0), k


def test_adam_constant_gradient_closed_form():
    """For a constant gradient the bias-corrected moments are exactly g and
    g^2, so every step moves each parameter by lr * g / (|g| + eps)."""
    rng = np.random.Generator(np.random.PCG64(11))
    p0 = rng.normal(0, 1, 50)
    g = rng.normal(0, 1e-2, 50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k in range(1, 6):
        p, m, v = OL.adam_step(p, m, v, g, k, lr=1e-3)
    np.testing.assert_allclose(p, p0 - 5 * 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)


def test_bf16_rounding_exact_values():
    one = 1.0
    u = 2.0 ** -7  # bf16 spacing at 1
    vals = np.array([one, one + u / 2, one + 3 * u / 2, one + u / 4, -2.0 - u, 3.0e38, 1.5e-39], np.float64)
    got = OL.bf16_round(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0             # halfway, ties to the even mantissa
    assert got[2] == one + 2 * u     # halfway, ties up to even
    assert got[3] == 1.0
    assert got[4] == -2.0            # spacing at 2 is 2u: -2 - u is halfway, even is -2
    assert np.isfinite(got[5]) and abs(got[5] / 3.0e38 - 1) < 2 ** -8
    assert abs(got[6] - 1.5e-39) <= 2.0 ** -133  # subnormal keeps 16 bits


def test_forward_wiring_hand_built_network():
    """W1 and W3 pick the first seven inputs and W2 is the identity, so the
    first seven logits are relu(x) + b3 and the rest are b3."""
    P = OL.unpack_params(np.zeros(OL.N_PARAMS))
    P["W1"][:7, :7] = np.eye(7)
    P["W2"][:] = np.eye(64)
    P["W3"][:7, :7] = np.eye(7)
    P["b3"][:] = np.arange(32) * 0.5
    params = OL.pack_params(P)
    x = np.array([[0.5, -1.0, 2.0, -0.25, 3.0, 0.0, 1.25], [-2.0, 1.0, -1.0, 4.0, -3.0, 0.75, -0.5]])
    z = OL.forward(params, x)
    want = np.tile(np.arange(32) * 0.5, (2, 1))
    want[:, :7] += np.maximum(x, 0.0)
    np.testing.assert_array_equal(z, want)
    np.testing.assert_array_equal(OL.forward(params, x, bf16=True), want)  # all values exact in bf16


def test_top3_order_and_mass():
    z = np.array([[0.0, 3.0, 1.0, 3.0, -1.0] + [-50.0] * 27])
    idx, mass = OL.top3(z)
    assert list(idx[0]) == [1, 3, 2]  # tie 1 vs 3 by index
    e = np.exp(z[0] - 3.0)
    assert abs(mass[0] - (e[1] + e[3] + e[2]) / e.sum()) < 1e-15


@pytest.fixture(scope="module")
def tiny_truth():
    from synth import barrel10, make_event
    det = barrel10()
    ev = make_event(det, 1, kind="tiny")
    return det, ev


def _full_table(g, mods):
    n_mod = g["center"].shape[0]
    sn, sr, sa = OL.neighbour_table(g, modules=mods)
    nxt = np.full((n_mod, OL.MAX_NEXT), -1, np.int32)
    reg = np.full((n_mod, OL.MAX_NEXT, OL.REG_U * OL.REG_V), -1, np.int32)
    anc = np.zeros((n_mod, OL.MAX_NEXT, 5))
    nxt[mods], reg[mods], anc[mods] = sn, sr, sa
    return nxt, reg, anc


def test_window_covers_truth_transitions(tiny_truth):
    """Particles from the origin (tiny event, pT 1-10 GeV): at every layer
    change of the truth trajectory the next layer is listed for the module
    left, and the module crossed there lies in the 32-cell window around
    the local helix's crossing of that layer's envelope."""
    det, ev = tiny_truth
    g = det.as_arrays()
    tr = ev.truth
    layer = g["layer"]
    nxt, reg, anc = _full_table(g, np.unique(tr.surface))
    n = ok = 0
    for k in range(len(tr.particle) - 1):
        if tr.particle[k] != tr.particle[k + 1]:
            continue
        m, m2 = int(tr.surface[k]), int(tr.surface[k + 1])
        if layer[m] == layer[m2]:
            continue
        n += 1
        s = np.nonzero(nxt[m] == layer[m2])[0]
        if len(s) == 0:
            continue
        d = tr.dir[k]
        p = [tr.loc[k, 0], tr.loc[k, 1], np.arctan2(d[1], d[0]), np.arccos(d[2]), tr.qop[k]]
        cr = OL.state_crossing(g, m, p, int(layer[m2]))
        if cr is None:
            continue
        ok += OL.window_label(g, int(layer[m2]), cr[0], anc[m, s[0]], reg[m, s[0]], m2) >= 0
    assert n > 500 and ok / n >= 0.995, (ok, n)


def test_region_invariants():
    """Anchors lie on the layer's envelope, beyond the module; every stored
    module belongs to the layer and sits in the cell its centre offset
    rounds to; a module appears at most once; and the module nearest to the
    anchor is the region's centre cell."""
    from synth import barrel_endcap
    det = barrel_endcap()
    g = det.as_arrays()
    rng = np.random.Generator(np.random.PCG64(5))
    mods = rng.choice(g["center"].shape[0], 300, replace=False)
    nxt, reg, anc = OL.neighbour_table(g, modules=mods)
    layer = g["layer"]
    c = g["center"].astype(np.float64)
    for i, m in enumerate(mods):
        for s in range(OL.MAX_NEXT):
            L = nxt[i, s]
            if L < 0:
                assert np.all(reg[i, s] == -1)
                continue
            assert L != layer[m]
            A = anc[i, s, :3]
            if g["layer_type"][L] == 0:
                assert abs(np.hypot(A[0], A[1]) - g["layer_pos"][L]) < 1e-9
            else:
                assert abs(A[2] - g["layer_pos"][L]) < 1e-9
            assert np.linalg.norm(A) > np.linalg.norm(c[m]) - np.hypot(*g["half"][m])
            pu, pv = anc[i, s, 3], anc[i, s, 4]
            assert 5.0 < pu < 25.0 and 20.0 < pv < 70.0
            ids = reg[i, s]
            k = np.nonzero(ids >= 0)[0]
            assert len(k) > 0 and len(set(ids[k])) == len(k)
            assert np.all(layer[ids[k]] == L)
            du, dv = OL.layer_coords(g, L, c[ids[k]], A)
            np.testing.assert_array_equal(OL._rnd(du / pu), k % OL.REG_U + OL.RU0)
            np.testing.assert_array_equal(OL._rnd(dv / pv), k // OL.REG_U + OL.RV0)
            mem = np.nonzero(layer == L)[0]
            du_all, dv_all = OL.layer_coords(g, L, c[mem], A)
            near = mem[np.argmin(du_all * du_all + dv_all * dv_all)]
            centre = (0 - OL.RV0) * OL.REG_U + (0 - OL.RU0)
            assert ids[centre] == near


def test_features_definition():
    """Straight line (no field) from a barrel module: the crossing of the
    next barrel's cylinder is the closed-form line/cylinder solution, the
    input's position is its fractional cell offset and the direction is the
    line's direction in the layer frame."""
    from synth import barrel_endcap
    det = barrel_endcap()
    g = det.as_arrays()
    l1 = np.nonzero(g["layer"] == 1)[0]
    m = int(l1[np.argmin(np.abs(g["center"][l1, 2]))])  # a central module: the next layer is a barrel
    nxt, reg, anc = OL.neighbour_table(g, modules=[m])
    L = int(nxt[0, 0])
    assert g["layer_type"][L] == 0
    p = np.array([2.0, -7.0, 0.3, 1.4, 0.8])
    X, Tx = OL.state_crossing(g, m, p, L, bfield=(0.0, 0.0, 0.0))
    rot = g["rot"].reshape(-1, 3, 3).astype(np.float64)
    P = g["center"][m].astype(np.float64) + p[0] * rot[m, 0] + p[1] * rot[m, 1]
    T = np.array([np.cos(p[2]) * np.sin(p[3]), np.sin(p[2]) * np.sin(p[3]), np.cos(p[3])])
    R = float(g["layer_pos"][L])
    a, b, cc = T[0] ** 2 + T[1] ** 2, P[0] * T[0] + P[1] * T[1], P[0] ** 2 + P[1] ** 2 - R * R
    s = (-b + np.sqrt(b * b - a * cc)) / a
    np.testing.assert_allclose(X, P + s * T, atol=1e-9)
    np.testing.assert_allclose(Tx, T, atol=1e-12)
    x = OL.features_at(g, L, X, Tx, p[4], anc[0, 0])
    A = anc[0, 0, :3]
    du = ((np.arctan2(X[1], X[0]) - np.arctan2(A[1], A[0]) + np.pi) % (2 * np.pi) - np.pi) * R
    qu = du / anc[0, 0, 3]
    assert abs(x[0] - (qu - np.floor(qu + 0.5))) < 1e-12 and -0.5 <= x[0] < 0.5
    qv = (X[2] - A[2]) / anc[0, 0, 4]
    assert abs(x[1] - (qv - np.floor(qv + 0.5))) < 1e-12
    r = np.hypot(X[0], X[1])
    np.testing.assert_allclose(x[2:5], [(-X[1] * T[0] + X[0] * T[1]) / r, T[2], (X[0] * T[0] + X[1] * T[1]) / r],
                               atol=1e-12)
    assert x[5] == p[4] and x[6] == L / g["layer_type"].shape[0]
    # the window's module ids are the region's cells around the crossing
    win = OL.window_modules(g, L, X, anc[0, 0], reg[0, 0])
    lab = OL.window_label(g, L, X, anc[0, 0], reg[0, 0], win[20])
    assert win[20] < 0 or lab == 20


def test_pairs_from_oracle_tracks(tiny_truth):
    """Pairs taken from the oracle's own tracks on the tiny event: the label
    points at the module of the next measurement in the window, the input is
    that of the measurement the pair starts from, and the per-measurement
    states end in the track's output state."""
    import oracle
    det, ev = tiny_truth
    g = det.as_arrays()
    inp = oracle.Inputs(g, (0, 0, 2.0), ev)
    r = oracle.ckf_find(inp, material_on=0)
    off, ms, mp = r["offsets"], r["meas_surface"], r["meas_params"]
    assert r["n_tracks"] > 90
    np.testing.assert_array_equal(mp[off[1:] - 1], r["params"])
    np.testing.assert_array_equal(ms[off[1:] - 1], r["last_surface"])
    nxt, reg, anc = _full_table(g, np.unique(ms))
    x, lab, trk, pos, dropped = OL.capture_pairs(g, nxt, reg, anc, off, ms, mp)
    layer = g["layer"]
    # one pair per measurement of the next layer after each change of layer
    want = 0
    for t in range(len(off) - 1):
        for i in range(off[t], off[t + 1] - 1):
            if layer[ms[i]] != layer[ms[i + 1]]:
                j = i + 1
                while j < off[t + 1] and layer[ms[j]] == layer[ms[i + 1]]:
                    want += 1
                    j += 1
    # drops: the next measurement lies beyond a hole, on a layer that is not next
    assert len(lab) + dropped == want and dropped <= 0.03 * want
    for k in range(len(lab)):
        m = ms[pos[k]]
        L2 = int(layer[ms[pos[k] + 1]])
        s = list(nxt[m]).index(L2)
        X, Tx = OL.state_crossing(g, m, mp[pos[k]], L2)
        mod = OL.window_modules(g, L2, X, anc[m, s], reg[m, s])[lab[k]]
        j = pos[k] + 1
        on_layer = []
        while j < off[trk[k] + 1] and layer[ms[j]] == L2:
            on_layer.append(ms[j])
            j += 1
        assert mod in on_layer
        np.testing.assert_array_equal(x[k], OL.features_at(g, L2, X, Tx, mp[pos[k]][4], anc[m, s]))
        assert off[trk[k]] <= pos[k] < off[trk[k] + 1] - 1


def test_bf16_gradient_mode_stays_close():
    """The bf16-rounding mode of the gradient (the precision of the matrix-core
    kernels) stays close to the FP64 gradient, and equals it when every
    rounded quantity is already a bf16 value (zero hidden layers' input)."""
    params, x, labels = _rand_problem(n=50, seed=8)
    _, g = OL.loss_and_grad(params, x, labels)
    _, gb = OL.loss_and_grad(params, x, labels, bf16=True)
    assert g @ gb / (np.linalg.norm(g) * np.linalg.norm(gb)) > 0.999
    P = OL.unpack_params(params)
    for k in ("W1", "W2", "W3"):
        P[k][:] = OL.bf16_round(P[k])
    P["W3"][:] = 0.0  # backpropagated gradients vanish below the output layer
    p2 = OL.pack_params(P)
    x2 = OL.bf16_round(np.zeros_like(x))
    l1, g1 = OL.loss_and_grad(p2, x2, labels)
    l2, g2 = OL.loss_and_grad(p2, x2, labels, bf16=True)
    G1, G2 = OL.unpack_params(g1), OL.unpack_params(g2)
    np.testing.assert_array_equal(G1["b3"], G2["b3"])
    assert l1 == l2
