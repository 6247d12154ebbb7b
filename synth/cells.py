"""Seeded synthetic detector cells (pixels and short strips) for clustering.

Each module is a grid of n0 x n1 cells whose pitch is the module's
measurement resolution times sqrt(12) (so that a one-cell cluster has the
resolution the track finder assumes), rounded to a whole number of cells.
A particle crossing deposits charge along its path through the 0.15 mm
sensor: the path's projection on the module plane is cut into 24 equal
pieces and each piece's charge (proportional to the path length) goes to the
cell it falls in.  Cells above threshold after Gaussian electronic noise are
read out; random noise cells are added; cells that two particles share are
merged (charges added, the larger contributor kept as truth).  Cells come
out in readout order: by (event, module), then row (c1), then column (c0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .detector import Detector

SENSOR_THICKNESS = 0.15   # mm of silicon
N_SAMPLES = 24            # pieces of the path projection
THRESHOLD = 0.12          # fraction of a normal-incidence crossing's charge
NOISE_SIGMA = 0.02
NOISE_CELLS = 2000        # mean number of random noise cells per event


def cell_grid(det: Detector):
    """(n0, n1) cells per module and the pitch (p0, p1) in mm, float32."""
    half = det.half.astype(np.float64)
    sig = det.sigma().astype(np.float64)
    n = np.maximum(1, np.rint(2.0 * half / (sig * np.sqrt(12.0)))).astype(np.int32)
    pitch = (2.0 * half / n).astype(np.float32)
    return n, pitch


@dataclass
class Cells:
    n_events: int
    n_surfaces: int
    offsets: np.ndarray    # (E*S + 1,) int32: cells of (event e, module s) are rows offsets[e*S+s]:offsets[e*S+s+1]
    c0: np.ndarray         # (n,) int32 column
    c1: np.ndarray         # (n,) int32 row
    q: np.ndarray          # (n,) float32 charge
    particle: np.ndarray   # (n,) int64 truth (largest contributor), -1 noise

    @property
    def n_cells(self):
        return int(self.c0.shape[0])


def make_cells(det: Detector, ev, rng_seed: int, noise_cells=NOISE_CELLS) -> Cells:
    """Cells of the truth crossings of a single event `ev` (synth.Event)."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    S = det.n_surfaces
    n, pitch = cell_grid(det)
    tr = ev.truth
    s = tr.surface.astype(np.int64)
    rot = det.rot.astype(np.float64)[s]          # rows u, v, n
    d = tr.dir.astype(np.float64)
    du, dv, dn = (np.einsum("ki,ki->k", rot[:, r], d) for r in range(3))
    dn = np.where(np.abs(dn) < 1e-3, np.copysign(1e-3, dn), dn)
    h = 0.5 * SENSOR_THICKNESS
    a0, a1 = tr.loc[:, 0] - h * du / dn, tr.loc[:, 1] - h * dv / dn
    b0, b1 = tr.loc[:, 0] + h * du / dn, tr.loc[:, 1] + h * dv / dn
    charge = 1.0 / np.abs(dn)                      # path length over the thickness
    t = (np.arange(N_SAMPLES) + 0.5) / N_SAMPLES
    x0 = a0[:, None] + (b0 - a0)[:, None] * t[None, :]
    x1 = a1[:, None] + (b1 - a1)[:, None] * t[None, :]
    half = det.half.astype(np.float64)[s]
    p = pitch.astype(np.float64)[s]
    i0 = np.floor((x0 + half[:, 0:1]) / p[:, 0:1]).astype(np.int64)
    i1 = np.floor((x1 + half[:, 1:2]) / p[:, 1:2]).astype(np.int64)
    inside = (i0 >= 0) & (i0 < n[s, 0:1]) & (i1 >= 0) & (i1 < n[s, 1:2])
    k = np.nonzero(inside)
    key = (s[k[0]] * 1024 + i1[k]) * 1024 + i0[k]
    part = tr.particle[k[0]].astype(np.int64)
    dq = (charge / N_SAMPLES)[k[0]]
    # charge per (cell, particle), then per cell with the larger contributor as truth
    up, inv = np.unique(key * (1 << 20) + part, return_inverse=True)
    qp = np.bincount(inv, weights=dq)
    ck, pk = up >> 20, up & ((1 << 20) - 1)
    cells, cinv = np.unique(ck, return_inverse=True)
    q = np.bincount(cinv, weights=qp)
    best = np.zeros(cells.size, np.int64)
    order = np.lexsort((-qp, cinv))
    first = order[np.r_[True, cinv[order][1:] != cinv[order][:-1]]]
    best[cinv[first]] = pk[first]
    q = q + rng.normal(0.0, NOISE_SIGMA, q.size)
    keep = q > THRESHOLD
    cells, q, best = cells[keep], q[keep], best[keep]
    # random noise cells
    nn = rng.poisson(noise_cells)
    ns = rng.integers(0, S, nn)
    nk = (ns * 1024 + rng.integers(0, n[ns, 1])) * 1024 + rng.integers(0, n[ns, 0])
    nq = rng.uniform(THRESHOLD, 1.0, nn)
    allk = np.concatenate([cells, nk])
    allq = np.concatenate([q, nq])
    allp = np.concatenate([best, np.full(nn, -1, np.int64)])
    uk, uinv = np.unique(allk, return_inverse=True)
    uq = np.bincount(uinv, weights=allq)
    up_ = np.full(uk.size, -1, np.int64)
    o = np.lexsort((-allq, uinv))
    f = o[np.r_[True, uinv[o][1:] != uinv[o][:-1]]]
    up_[uinv[f]] = allp[f]
    mod = uk // (1024 * 1024)
    c1 = (uk // 1024) % 1024
    c0 = uk % 1024
    offsets = np.zeros(S + 1, np.int64)
    np.add.at(offsets, mod + 1, 1)
    offsets = np.cumsum(offsets)
    return Cells(1, S, offsets.astype(np.int32), c0.astype(np.int32), c1.astype(np.int32), uq.astype(np.float32),
                 up_)


def concat_cells(cs) -> Cells:
    S = cs[0].n_surfaces
    offs, base = [np.zeros(1, np.int64)], 0
    for c in cs:
        offs.append(c.offsets[1:].astype(np.int64) + base)
        base += c.n_cells
    return Cells(sum(c.n_events for c in cs), S, np.concatenate(offs).astype(np.int32),
                 np.concatenate([c.c0 for c in cs]), np.concatenate([c.c1 for c in cs]),
                 np.concatenate([c.q for c in cs]), np.concatenate([c.particle for c in cs]))
