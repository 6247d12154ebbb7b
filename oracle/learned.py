"""FP64 oracle of the learned next-module proposal and its training.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain numpy in
float64, written from the definitions, sharing nothing with the GPU library.

What is defined here:

* the neighbour table of a detector: for every module m the (at most three)
  layers a straight ray from the origin through m meets next, and for each
  such layer L' the anchor (where the first ray meeting L' crosses its
  envelope), the layer's module pitches there, and a 24 x 8 region of
  cells in the layer's curvilinear coordinates around the anchor, each cell
  holding the L' module whose centre falls in it;
* the proposal window: the 8 x 4 cells around the cell where the local
  helix from the state on m crosses L''s envelope; the 7-number input of
  the network is that crossing's fractional position in its cell, the
  direction there in the layer's local frame, q/p and L';
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


WIN_U, WIN_V = 8, 4            # the 32 network outputs: cells iu in [-4, 3] x iv in [-2, 1] around the crossing
WU0, WV0 = -4, -2
REG_U, REG_V = 24, 8           # the stored region: cells iu in [-12, 11] x iv in [-4, 3] around the anchor
RU0, RV0 = -12, -4


def _rnd(x):
    return np.floor(x + 0.5)


def _wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def layer_coords(geom, L, X, A):
    """Curvilinear offsets of points X [..., 3] from the anchor A on layer L:
    barrels (R dphi, dz) with R the layer radius, disks (r dphi, dr) with r
    the point's own radius."""
    X = np.asarray(X, np.float64)
    dphi = _wrap(np.arctan2(X[..., 1], X[..., 0]) - np.arctan2(A[1], A[0]))
    rX = np.hypot(X[..., 0], X[..., 1])
    if int(geom["layer_type"][L]) == 0:
        return dphi * float(geom["layer_pos"][L]), X[..., 2] - A[2]
    return dphi * rX, rX - np.hypot(A[0], A[1])


def _cells(geom, L, A):
    """Pitches and the stored region of layer L around anchor A: the pitch
    along u is the smallest positive u-offset between the module nearest to
    A (ties by id) and another module of its row (|dv| < its half length v),
    the pitch along v the smallest positive v-offset to a module of its
    column (|du| < half the u pitch), else the module's full lengths; a
    module sits in cell (round(du/pu), round(dv/pv)) of its centre's offset
    from A, and each cell of the 24 x 8 region keeps the module nearest to
    the cell's centre (ties by id)."""
    layer = np.asarray(geom["layer"])
    c = np.asarray(geom["center"], np.float64)
    half = np.asarray(geom["half"], np.float64)
    mem = np.nonzero(layer == L)[0]
    du, dv = layer_coords(geom, L, c[mem], A)
    d2 = du * du + dv * dv
    a = int(np.lexsort((mem, d2))[0])
    ou, ov = du - du[a], dv - dv[a]
    row = (np.abs(ov) < half[mem[a], 1]) & (ou > 1e-3)
    pu = float(ou[row].min()) if row.any() else 2.0 * half[mem[a], 0]
    col = (np.abs(ou) < 0.5 * pu) & (ov > 1e-3)
    pv = float(ov[col].min()) if col.any() else 2.0 * half[mem[a], 1]
    iu, iv = _rnd(du / pu), _rnd(dv / pv)
    region = np.full(REG_U * REG_V, -1, np.int32)
    best = np.full(REG_U * REG_V, np.inf)
    ok = (iu >= RU0) & (iu < RU0 + REG_U) & (iv >= RV0) & (iv < RV0 + REG_V)
    for j in np.nonzero(ok)[0]:
        k = int((iv[j] - RV0) * REG_U + (iu[j] - RU0))
        eu, ev = du[j] - iu[j] * pu, dv[j] - iv[j] * pv
        dist = eu * eu + ev * ev
        m = int(mem[j])
        if dist < best[k] or (dist == best[k] and m < region[k]):
            best[k], region[k] = dist, m
    return pu, pv, region


def neighbour_table(geom, modules=None):
    """For the given modules (all by default): next layers [n, 3], the stored
    cell regions [n, 3, 192] and the anchors with pitches [n, 3, 5] =
    (anchor x, y, z, pitch u, pitch v) of each (module, next layer); -1 pads
    the regions (and the layers)."""
    n_mod = np.asarray(geom["center"]).shape[0]
    mods = np.arange(n_mod) if modules is None else np.asarray(modules)
    layer = np.asarray(geom["layer"])
    pts = _ray_points(geom)[mods]
    tm = np.linalg.norm(pts, axis=-1)
    dirs = pts / tm[..., None]
    t = _ray_crossings(geom, dirs)  # (k, 5, L)
    own = layer[mods]
    t[np.arange(len(mods))[:, None], :, own[:, None]] = np.inf
    t = np.where(t > tm[..., None], t, np.inf)
    first = np.argmin(t, axis=-1)  # (k, 5)
    hit = np.isfinite(np.take_along_axis(t, first[..., None], -1)[..., 0])
    nxt = np.full((len(mods), MAX_NEXT), -1, np.int32)
    reg = np.full((len(mods), MAX_NEXT, REG_U * REG_V), -1, np.int32)
    anc = np.zeros((len(mods), MAX_NEXT, 5))
    for i in range(len(mods)):
        k = 0
        for r in range(5):
            if not hit[i, r]:
                continue
            L = int(first[i, r])
            if L in nxt[i, :k] or k == MAX_NEXT:
                continue
            nxt[i, k] = L
            A = t[i, r, L] * dirs[i, r]
            pu, pv, region = _cells(geom, L, A)
            anc[i, k] = (A[0], A[1], A[2], pu, pv)
            reg[i, k] = region
            k += 1
    return nxt, reg, anc


# ---------------------------------------------------------------------------
# Network input


def _helix_layer_crossing(P, T, qop, B, ltype, pos):
    """First positive-path crossing of the local helix (field B at P) with a
    barrel layer's cylinder r = pos or a disk layer's plane z = pos: Newton
    from the straight-line estimate (the navigation's own definition).
    Returns (s, point, direction) or None."""
    kappa = 2.99792458e-4
    bm = np.linalg.norm(B)
    bhat = B / bm if bm > 0 else np.array([0.0, 0.0, 1.0])
    om = kappa * qop * bm
    tpar = T @ bhat
    tperp = T - tpar * bhat
    w = np.cross(T, bhat)

    def at(s):
        a = om * s
        if abs(a) < 1e-4:
            S = s * (1 - a * a / 6.0)
            Cc = s * (0.5 * a) * (1 - a * a / 12.0)
        else:
            S = np.sin(a) / om
            Cc = 2.0 * np.sin(0.5 * a) ** 2 / om
        return P + tpar * s * bhat + S * tperp + Cc * w, tpar * bhat + np.cos(a) * tperp + np.sin(a) * w

    if ltype == 0:
        a = T[0] ** 2 + T[1] ** 2
        b = P[0] * T[0] + P[1] * T[1]
        c = P[0] ** 2 + P[1] ** 2 - pos * pos
        if a < 1e-12 or b * b - a * c < 0:
            return None
        s = (-b + np.sqrt(b * b - a * c)) / a
        if not s > 0:
            return None
        for _ in range(20):
            p, t = at(s)
            g = p[0] ** 2 + p[1] ** 2 - pos * pos
            gp = 2.0 * (p[0] * t[0] + p[1] * t[1])
            if not gp > 0:
                return None
            ds = g / gp
            s -= ds
            if abs(ds) < 1e-4:
                break
        if not s > 0:
            return None
        p, t = at(s)
        if abs(np.hypot(p[0], p[1]) - pos) > 1e-3:
            return None
        return s, p, t
    if abs(T[2]) < 1e-12:
        return None
    s = (pos - P[2]) / T[2]
    if not s > 0:
        return None
    for _ in range(20):
        p, t = at(s)
        if abs(t[2]) < 1e-12:
            return None
        ds = (p[2] - pos) / t[2]
        s -= ds
        if abs(ds) < 1e-4:
            break
    if not s > 0:
        return None
    p, t = at(s)
    return s, p, t


def crossing_window(geom, L, X, anc):
    """Centre cell (iu, iv) of the proposal window for a crossing X of layer
    L and the fractional position of X in it (each in [-1/2, 1/2))."""
    du, dv = layer_coords(geom, L, X, anc[:3])
    qu, qv = du / anc[3], dv / anc[4]
    iu, iv = _rnd(qu), _rnd(qv)
    return int(iu), int(iv), qu - iu, qv - iv


def features_at(geom, L, X, Tx, qop, anc):
    """Network input for a trajectory crossing layer L's envelope at X with
    direction Tx: its fractional position in the centre cell, the direction
    in the layer's local frame (phi-hat, then z-hat and r-hat for barrels,
    r-hat and z-hat for disks), q/p in 1/GeV, L / number of layers."""
    n_layers = np.asarray(geom["layer_type"]).shape[0]
    _, _, fu, fv = crossing_window(geom, L, X, anc)
    r = np.hypot(X[0], X[1])
    ph = np.array([-X[1] / r, X[0] / r, 0.0])
    rh = np.array([X[0] / r, X[1] / r, 0.0])
    zh = np.array([0.0, 0.0, 1.0])
    if int(geom["layer_type"][L]) == 0:
        tv, tn = Tx @ zh, Tx @ rh
    else:
        tv, tn = Tx @ rh, Tx @ zh
    return np.array([fu, fv, Tx @ ph, tv, tn, qop, L / n_layers])


def window_label(geom, L, X, anc, region, module):
    """Position (0..31) of `module` in the proposal window centred on the
    crossing X, or -1 when it is not in the stored region or the window."""
    iu, iv, _, _ = crossing_window(geom, L, X, anc)
    hits = np.nonzero(region == module)[0]
    if len(hits) == 0:
        return -1
    ku, kv = hits[0] % REG_U + RU0, hits[0] // REG_U + RV0
    wu, wv = ku - iu - WU0, kv - iv - WV0
    if not (0 <= wu < WIN_U and 0 <= wv < WIN_V):
        return -1
    return int(wv * WIN_U + wu)


def window_modules(geom, L, X, anc, region):
    """The 32 window entries (module ids, -1 outside the region or empty)
    around the crossing X, in output order."""
    iu, iv, _, _ = crossing_window(geom, L, X, anc)
    out = np.full(WIN_U * WIN_V, -1, np.int32)
    for k in range(WIN_U * WIN_V):
        cu, cv = iu + WU0 + k % WIN_U, iv + WV0 + k // WIN_U
        if RU0 <= cu < RU0 + REG_U and RV0 <= cv < RV0 + REG_V:
            out[k] = region[(cv - RV0) * REG_U + (cu - RU0)]
    return out


def state_crossing(geom, surface, params, L, bfield=(0.0, 0.0, 2.0)):
    """Where the local helix of the bound state on `surface` crosses layer
    L's envelope (point, direction), or None."""
    c = np.asarray(geom["center"], np.float64)
    rot = np.asarray(geom["rot"], np.float64).reshape(-1, 3, 3)
    p = np.asarray(params, np.float64)
    P = c[surface] + p[0] * rot[surface, 0] + p[1] * rot[surface, 1]
    T = np.array([np.cos(p[2]) * np.sin(p[3]), np.sin(p[2]) * np.sin(p[3]), np.cos(p[3])])
    hx = _helix_layer_crossing(P, T, p[4], np.asarray(bfield, np.float64), int(geom["layer_type"][L]),
                               float(geom["layer_pos"][L]))
    return None if hx is None else (hx[1], hx[2])


def capture_pairs(geom, nxt, reg, anc, offsets, meas_surface, meas_params, bfield=(0.0, 0.0, 2.0)):
    """Training pairs from found tracks (CSR `offsets` over the measurements,
    each with its module and filtered parameters).  Returns (x [k, 7],
    label [k], track [k], position [k], n_dropped); pairs in track order, then
    measurement order.  At each change of layer, the state at the last
    measurement of the layer gives the input (through its helix crossing of
    the next measurement's layer), and every measurement of the track on
    that layer (overlapping modules give several) gives one pair with its
    module's place in the window as the label; such a pair is dropped when
    the layer is not listed for the module, the helix misses the envelope,
    or the module is outside the window."""
    layer = np.asarray(geom["layer"])
    xs, labels, trk, posn, dropped = [], [], [], [], 0
    for t in range(len(offsets) - 1):
        for i in range(offsets[t], offsets[t + 1] - 1):
            m = int(meas_surface[i])
            L2 = int(layer[meas_surface[i + 1]])
            if L2 == layer[m]:
                continue
            j_end = i + 1
            while j_end < offsets[t + 1] and layer[meas_surface[j_end]] == L2:
                j_end += 1
            slots = np.nonzero(nxt[m] == L2)[0]
            cr = state_crossing(geom, m, meas_params[i], L2, bfield) if len(slots) else None
            for j in range(i + 1, j_end):
                m2 = int(meas_surface[j])
                lab = -1
                if cr is not None:
                    s = slots[0]
                    lab = window_label(geom, L2, cr[0], anc[m, s], reg[m, s], m2)
                if lab < 0:
                    dropped += 1
                    continue
                xs.append(features_at(geom, L2, cr[0], cr[1], float(meas_params[i][4]), anc[m, s]))
                labels.append(lab)
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
