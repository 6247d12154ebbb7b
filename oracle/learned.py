"""FP64 oracle of the learned next-module proposal and its training.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain numpy in
float64, written from the definitions, sharing nothing with the GPU library.

What is defined here:

* the neighbour table of a detector: for every module m the (at most three)
  layers a straight ray from the origin through m meets next, and for each
  such layer L' the 32 modules of L' whose centres are nearest to where the
  ray through m's centre (or, if that ray meets another layer first, the
  first corner ray that meets L') crosses L''s envelope, ties by id;
* the 7-number state that the network sees on module m when it asks for
  layer L';
* the (state, label) pairs taken from found tracks: at every change of layer
  between consecutive measurements, the state at the last measurement of the
  layer and the position of the next measurement's module in the table;
* the network 7 -> 64 -> 64 -> 32 (ReLU, softmax), its mean cross-entropy
  loss and gradient, and one Adam step.

The proposal and its training are not in the paper: the paper's navigation
searches the detector geometry (section 2); the learned form replaces only
the module lookup and keeps that search as its fallback.
"""
from __future__ import annotations

import numpy as np

K_NEIGH = 32   # modules per (module, next layer)
MAX_NEXT = 3   # next layers per module
N_IN, N_H, N_OUT = 7, 64, 32

# flat parameter layout: W1 [64][7], b1 [64], W2 [64][64], b2 [64], W3 [32][64], b3 [32]
_SHAPES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
           ("W3", (N_OUT, N_H)), ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in _SHAPES)  # 6752


def unpack_params(flat):
    flat = np.asarray(flat, np.float64)
    assert flat.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in _SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack_params(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in _SHAPES])


def init_params(seed: int):
    """He-uniform weights, zero biases, from numpy's PCG64(seed) (float32 values)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {}
    for name, shape in _SHAPES:
        if name.startswith("W"):
            fan_in = shape[1]
            lim = np.sqrt(6.0 / fan_in)
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    return pack_params(d).astype(np.float32)


# ---------------------------------------------------------------------------
# Neighbour table


def _ray_crossings(geom, dirs):
    """Path t along unit rays `dirs` (..., 3) from the origin to every layer's
    envelope, inf where the ray misses it (outside the extent or backwards)."""
    lt = np.asarray(geom["layer_type"])
    pos = np.asarray(geom["layer_pos"], np.float64)
    lo = np.asarray(geom["layer_lo"], np.float64)
    hi = np.asarray(geom["layer_hi"], np.float64)
    dperp = np.hypot(dirs[..., 0], dirs[..., 1])[..., None]
    dz = dirs[..., 2][..., None]
    with np.errstate(divide="ignore", invalid="ignore"):
        t_cyl = pos / dperp
        z_cyl = t_cyl * dz
        ok_cyl = (dperp > 0) & (z_cyl >= lo) & (z_cyl <= hi)
        t_dsk = pos / dz
        r_dsk = t_dsk * dperp
        ok_dsk = (dz != 0) & (t_dsk > 0) & (r_dsk >= lo) & (r_dsk <= hi)
    barrel = lt == 0
    t = np.where(barrel, np.where(ok_cyl, t_cyl, np.inf), np.where(ok_dsk, t_dsk, np.inf))
    return t


def _ray_points(geom):
    """Per module: the 5 ray targets (centre, then corners (-,-), (+,-), (-,+), (+,+))."""
    c = np.asarray(geom["center"], np.float64)
    rot = np.asarray(geom["rot"], np.float64).reshape(-1, 3, 3)
    u, v = rot[:, 0], rot[:, 1]
    h = np.asarray(geom["half"], np.float64)
    pts = [c]
    for s1, s0 in ((-1, -1), (-1, 1), (1, -1), (1, 1)):
        pts.append(c + s0 * h[:, :1] * u + s1 * h[:, 1:2] * v)
    return np.stack(pts, axis=1)  # (n, 5, 3)


def neighbour_table(geom, modules=None):
    """(next_layers [n, 3], neighbours [n, 3, 32]) for the given modules
    (all by default); -1 pads."""
    n_mod = np.asarray(geom["center"]).shape[0]
    mods = np.arange(n_mod) if modules is None else np.asarray(modules)
    layer = np.asarray(geom["layer"])
    centers = np.asarray(geom["center"], np.float64)
    pts = _ray_points(geom)[mods]
    tm = np.linalg.norm(pts, axis=-1)
    dirs = pts / tm[..., None]
    t = _ray_crossings(geom, dirs)  # (k, 5, L)
    own = layer[mods]
    n_layers = t.shape[-1]
    t[np.arange(len(mods))[:, None], :, own[:, None]] = np.inf
    t = np.where(t > tm[..., None], t, np.inf)
    first = np.argmin(t, axis=-1)  # (k, 5)
    hit = np.isfinite(np.take_along_axis(t, first[..., None], -1)[..., 0])
    nxt = np.full((len(mods), MAX_NEXT), -1, np.int32)
    nbr = np.full((len(mods), MAX_NEXT, K_NEIGH), -1, np.int32)
    anchors = np.zeros((len(mods), MAX_NEXT, 3))
    for i in range(len(mods)):
        k = 0
        for r in range(5):
            if not hit[i, r]:
                continue
            L = int(first[i, r])
            if L in nxt[i, :k] or k == MAX_NEXT:
                continue
            nxt[i, k] = L
            anchors[i, k] = t[i, r, L] * dirs[i, r]
            k += 1
    by_layer = [np.nonzero(layer == L)[0] for L in range(n_layers)]
    for L in range(n_layers):
        sel = np.nonzero(nxt == L)
        if len(sel[0]) == 0:
            continue
        cand = by_layer[L]
        X = anchors[sel]  # (q, 3)
        d = centers[cand][None, :, :] - X[:, None, :]
        d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        order = np.lexsort((np.broadcast_to(cand, d2.shape), d2), axis=-1)[:, :K_NEIGH]
        nbr[sel[0], sel[1], :order.shape[1]] = cand[order]
    return nxt, nbr, anchors


# ---------------------------------------------------------------------------
# Network input


def features(geom, surface, params, target_layer):
    """State on module `surface` with bound params (loc0, loc1, phi, theta, q/p)
    asking for layer `target_layer`: loc0/10, loc1/30, the unit direction in
    the module frame (u, v, n), q/p in 1/GeV, target layer / number of layers."""
    surface = np.asarray(surface)
    p = np.asarray(params, np.float64).reshape(-1, 5)
    rot = np.asarray(geom["rot"], np.float64).reshape(-1, 3, 3)[surface]
    n_layers = np.asarray(geom["layer_type"]).shape[0]
    ph, th = p[:, 2], p[:, 3]
    T = np.stack([np.cos(ph) * np.sin(th), np.sin(ph) * np.sin(th), np.cos(th)], axis=-1)
    loc_dir = np.einsum("kij,kj->ki", rot, T)
    x = np.empty((p.shape[0], N_IN))
    x[:, 0] = p[:, 0] / 10.0
    x[:, 1] = p[:, 1] / 30.0
    x[:, 2:5] = loc_dir
    x[:, 5] = p[:, 4]
    x[:, 6] = np.asarray(target_layer, np.float64) / n_layers
    return x


def capture_pairs(geom, nxt, nbr, offsets, meas_surface, meas_params):
    """Training pairs from found tracks (CSR `offsets` over the measurements,
    each with its module and filtered parameters).  Returns (x [k, 7],
    label [k], track [k], position [k], n_dropped); pairs in track order, then
    measurement order."""
    layer = np.asarray(geom["layer"])
    xs, labels, trk, posn, dropped = [], [], [], [], 0
    for t in range(len(offsets) - 1):
        for i in range(offsets[t], offsets[t + 1] - 1):
            m, m2 = int(meas_surface[i]), int(meas_surface[i + 1])
            if layer[m2] == layer[m]:
                continue
            L2 = int(layer[m2])
            slots = np.nonzero(nxt[m] == L2)[0]
            if len(slots) == 0:
                dropped += 1
                continue
            pos = np.nonzero(nbr[m, slots[0]] == m2)[0]
            if len(pos) == 0:
                dropped += 1
                continue
            xs.append(features(geom, [m], meas_params[i], [L2])[0])
            labels.append(int(pos[0]))
            trk.append(t)
            posn.append(i)
    x = np.array(xs).reshape(-1, N_IN)
    return x, np.array(labels, np.int32), np.array(trk, np.int32), np.array(posn, np.int64), dropped


# ---------------------------------------------------------------------------
# Network, loss, gradient, Adam


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, np.float32).copy()
    u = f.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return f.astype(np.float64)


def forward(params, x, bf16=False):
    """Logits [n, 32].  bf16=True rounds the weights, the input and both hidden
    activations to bfloat16 where a bf16 matrix-core evaluation does (biases
    and sums stay wide)."""
    P = unpack_params(params)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    x = r(x)
    z1 = x @ r(P["W1"]).T + P["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(P["W2"]).T + P["b2"]
    h2 = r(np.maximum(z2, 0.0))
    return h2 @ r(P["W3"]).T + P["b3"]


def softmax(z):
    z = z - z.max(axis=-1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=-1, keepdims=True)


def loss_and_grad(params, x, labels, bf16=False):
    """Mean softmax cross-entropy over the rows and its gradient (flat, FP64)
    by reverse-mode differentiation of the three layers.  bf16=True rounds
    to bfloat16 where a bf16 matrix-core evaluation does: the weights, the
    input, both hidden activations and the three backpropagated
    pre-activation gradients where they enter products (bias gradients use
    the unrounded ones); the ReLU derivative is then taken from the rounded
    activation."""
    P = unpack_params(params)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    x = r(x)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    n = x.shape[0]
    z1 = x @ W1.T + P["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + P["b2"]
    h2 = r(np.maximum(z2, 0.0))
    z3 = h2 @ W3.T + P["b3"]
    p = softmax(z3)
    rows = np.arange(n)
    loss = -np.mean(np.log(p[rows, labels]))
    dz3 = p.copy()
    dz3[rows, labels] -= 1.0
    dz3 /= n
    g = {"W3": r(dz3).T @ h2, "b3": dz3.sum(0)}
    dz2 = (r(dz3) @ W3) * ((h2 > 0) if bf16 else (z2 > 0))
    g["W2"], g["b2"] = r(dz2).T @ h1, dz2.sum(0)
    dz1 = (r(dz2) @ W2) * ((h1 > 0) if bf16 else (z1 > 0))
    g["W1"], g["b1"] = r(dz1).T @ x, dz1.sum(0)
    return loss, pack_params(g)


def adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, with bias correction); `step` counts
    from 1.  Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def top3(logits):
    """(indices [n, 3], summed probability [n]) of the three most probable
    outputs, ties by index."""
    p = softmax(np.asarray(logits, np.float64))
    idx = np.argsort(-p, axis=-1, kind="stable")[:, :3]
    return idx, np.take_along_axis(p, idx, -1).sum(-1)
