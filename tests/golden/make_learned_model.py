"""Writes ``learned_model.txt``: next-module network parameters trained by the
FP64 oracle alone, for the learned-search parity tests.

Nothing here touches the GPU library.  The training pairs come from the
oracle's own plain track finding on four mu = 200 events of the barrel +
endcap detector (generator seeds 5000..5003), captured with the oracle's
pair definition (``oracle.learned.capture_pairs``: at each change of layer,
the filtered state at the last measurement of the layer and the window cell
of the next measurement's module).  The network 7 -> 64 -> 64 -> 32 is
trained with the oracle's FP64 loss, gradient and Adam (He-uniform start
from PCG64(7), batch 2048, lr 1e-3, 8 epochs, rows shuffled by PCG64(8)
every epoch).  The parameters are written as FP32 values, one per line, in
the order W1 [64][7], b1, W2 [64][64], b2, W3 [32][64], b3.

Run from the repository root:  python tests/golden/make_learned_model.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import learned as OL  # noqa: E402
from synth import barrel_endcap, make_event  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_model.txt")
EVENTS = (5000, 5001, 5002, 5003)


def pairs_of_event(det, g, seed):
    ev = make_event(det, seed, mu=200)
    r = oracle.ckf_find(oracle.Inputs(g, (0, 0, 2.0), ev))
    mods = np.unique(r["meas_surface"])
    n_mod = g["center"].shape[0]
    sn, sr, sa = OL.neighbour_table(g, modules=mods)
    nxt = np.full((n_mod, 3), -1, np.int32)
    reg = np.full((n_mod, 3, 192), -1, np.int32)
    anc = np.zeros((n_mod, 3, 5))
    nxt[mods], reg[mods], anc[mods] = sn, sr, sa
    x, lab, _, _, dropped = OL.capture_pairs(g, nxt, reg, anc, r["offsets"], r["meas_surface"], r["meas_params"])
    return x, lab, dropped


def main():
    oracle.build(force=not os.path.exists(oracle.LIB))
    det = barrel_endcap()
    g = det.as_arrays()
    xs, ls = [], []
    for s in EVENTS:
        t = time.time()
        x, lab, dropped = pairs_of_event(det, g, s)
        print(f"event {s}: {len(lab)} pairs, {dropped} dropped ({time.time() - t:.0f} s)", flush=True)
        xs.append(x)
        ls.append(lab)
    x = np.concatenate(xs)
    lab = np.concatenate(ls)
    n = len(lab)
    n_val = n // 10
    val = slice(n - n_val, n)
    tr = np.arange(n - n_val)
    params = OL.init_params(7).astype(np.float64)
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    rng = np.random.Generator(np.random.PCG64(8))
    step = 0
    for ep in range(8):
        perm = rng.permutation(tr)
        for b0 in range(0, len(perm), 2048):
            rows = perm[b0:b0 + 2048]
            loss, grad = OL.loss_and_grad(params, x[rows], lab[rows])
            step += 1
            params, m, v = OL.adam_step(params, m, v, grad, step)
        z = OL.forward(params, x[val])
        idx, mass = OL.top3(z)
        top3 = np.mean(np.any(idx == lab[val][:, None], axis=1))
        print(f"epoch {ep}: loss {loss:.4f}, validation top-3 {top3:.4f}, "
              f"rows with top-3 mass >= 0.95: {np.mean(mass >= 0.95):.3f}", flush=True)
    np.savetxt(OUT, params.astype(np.float32), fmt="%.9g")
    print(f"wrote {OUT} ({n} pairs, {step} Adam steps)")


if __name__ == "__main__":
    main()
