"""Training of the learned next-module proposal on the GPU.

Pairs (network input at the local helix's crossing of the next layer,
position of the next measurement's module in the window around it) come
from the plain track finder's own output (ckf_capture_pairs);
the network is trained by the library's kernels (ckf_mlp_grad on the bf16
matrix cores, ckf_mlp_adam), minibatches gathered on the device through a
row-index array.  Host code here only draws the seeded initial weights and
the epoch permutations and loops over launches.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from . import (Finder, Model, MlpWorkspace, _abi, capture_pairs, config, launch, mlp_adam, mlp_forward,
               mlp_grad)

N_PARAMS = _abi.MLP_PARAMS


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)) and zero biases, drawn from
    numpy's PCG64(seed), in the parameter order W1 [64][7], b1, W2 [64][64],
    b2, W3 [32][64], b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for out_dim, in_dim in ((64, 7), (64, 64), (32, 64)):
        lim = np.sqrt(6.0 / in_dim)
        parts.append(rng.uniform(-lim, lim, size=out_dim * in_dim))
        parts.append(np.zeros(out_dim))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == N_PARAMS
    return p


def make_pairs(geometry, field, batch, cfg=None, launch_cfg=None, stream=None):
    """Run the plain track finder on `batch` and capture its training pairs.
    Returns (x [k, 7], label [k]) device tensors, the number of tracks and
    the number of dropped pairs."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        f = Finder(geometry, field, batch, cfg, launch_cfg, counters=False, meas_states=True)
        f.enqueue(s)
        r = f.result()
        cap = int(r["offsets"][-1]) if r["n_tracks"] > 0 else 1
        x, lab, _, n_pairs, dropped = capture_pairs(geometry, field, f.out, cap, s)
        return x.clone(), lab.clone(), r["n_tracks"], dropped


@dataclass
class TrainLog:
    epochs: int = 0
    steps: int = 0
    loss: list = field(default_factory=list)      # mean training loss per epoch
    val_top1: float = 0.0
    val_top3: float = 0.0                         # label among the three most probable
    val_confident: float = 0.0                    # fraction with summed top-3 probability >= min_prob
    val_confident_right: float = 0.0             # ... of which the label is among the three


def train(x, labels, epochs=20, batch=4096, lr=1e-3, seed=0, val_frac=0.1, min_prob=0.95, stream=None,
          verbose=False):
    """Adam on the mean cross-entropy; returns (params [6752] float32 device
    tensor, TrainLog).  A fixed split (seeded) holds out val_frac of the
    pairs for the validation figures."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):  # the library calls and the torch ops share one stream
        return _train(x, labels, epochs, batch, lr, seed, val_frac, min_prob, s, verbose)


def _train(x, labels, epochs, batch, lr, seed, val_frac, min_prob, stream, verbose):
    import torch
    dev = x.device
    n = int(x.shape[0])
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(n)
    n_val = int(round(val_frac * n))
    val_idx, tr_idx = order[:n_val], order[n_val:]
    params = torch.as_tensor(init_params(seed), device=dev).contiguous()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = MlpWorkspace(batch, dev)
    log = TrainLog()
    step = 0
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(tr_idx).astype(np.int32), device=dev)
        ep_loss = torch.zeros(1, dtype=torch.float32, device=dev)
        nb = 0
        for b0 in range(0, len(tr_idx), batch):
            k = min(batch, len(tr_idx) - b0)
            mlp_grad(params, x, labels, rows=perm.data_ptr() + 4 * b0, n=k, workspace=ws, grad=grad, loss=loss,
                     stream=stream)
            step += 1
            mlp_adam(params, m, v, grad, step, lr=lr, stream=stream)
            ep_loss += loss
            nb += 1
        log.loss.append(float(ep_loss.item()) / max(1, nb))
        if verbose:
            print(f"# epoch {ep}: loss {log.loss[-1]:.4f}", flush=True)
    log.epochs, log.steps = epochs, step
    if n_val > 0:
        model = Model(params, stream)
        vi = torch.as_tensor(val_idx, device=dev)
        z = mlp_forward(model, x[vi].contiguous(), stream).double()
        p = torch.softmax(z, dim=1)
        top = torch.topk(p, 3, dim=1)
        lab = labels[vi].long()
        hit3 = (top.indices == lab[:, None]).any(dim=1)
        conf = top.values.sum(dim=1) >= min_prob
        log.val_top1 = float((top.indices[:, 0] == lab).double().mean())
        log.val_top3 = float(hit3.double().mean())
        log.val_confident = float(conf.double().mean())
        log.val_confident_right = float((hit3 & conf).double().sum() / max(1, int(conf.sum())))
    return params, log


def train_from_batches(geometry, field, batches, cfg=None, launch_cfg=None, min_pairs=0, stream=None, **kw):
    """Pairs from each batch in turn (until at least min_pairs), then train.
    Returns (params, TrainLog, info dict)."""
    import torch
    xs, ls, n_tracks, dropped = [], [], 0, 0
    for b in batches:
        x, lab, nt, dr = make_pairs(geometry, field, b, cfg, launch_cfg, stream)
        xs.append(x)
        ls.append(lab)
        n_tracks += nt
        dropped += dr
        if min_pairs and sum(int(t.shape[0]) for t in xs) >= min_pairs:
            break
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        x = torch.cat(xs).contiguous()
        lab = torch.cat(ls).contiguous()
    params, log = train(x, lab, stream=s, **kw)
    return params, log, dict(pairs=int(x.shape[0]), dropped=dropped, tracks=n_tracks)
