"""Oracle of cell clustering and measurement formation.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain Python in
float64, written from the definitions below and sharing nothing with the GPU
library.

The paper (section 2) starts the chain with hit clustering: the activated
cells of a sensor are grouped into clusters by a connected component
analysis, and each cluster's weighted centroid and its error make a
measurement, whose position in global coordinates is a spacepoint.  The
readings:

* two cells of the same module (and event) are connected when they touch,
  sides or corners (|dc0| <= 1 and |dc1| <= 1); clusters are the connected
  components;
* a cluster is named by its first cell in readout order (row c1, then
  column c0); a module's clusters are taken in that order;
* the measurement is the charge-weighted mean of the cluster's cell centres
  in local coordinates: with the sums W = sum q and X = sum q (c + 1/2) over
  the cluster's cells (in cell units), loc = pitch X / W - half length; its
  variances are pitch^2 / 12;
* the spacepoint is centre + loc0 u + loc1 v of the module.
"""
from __future__ import annotations

import numpy as np


def spacepoints(geom, surface, loc):
    """Global positions centre + loc0 u + loc1 v (float64) of points with
    local positions loc [n, 2] on modules surface [n] of the geometry
    (as_arrays()): the spacepoint definition above."""
    rot = geom["rot"].astype(np.float64).reshape(-1, 3, 3)
    centre = geom["center"].astype(np.float64)
    s = np.asarray(surface)
    loc = np.asarray(loc, np.float64)
    return centre[s] + loc[:, 0:1] * rot[s, 0] + loc[:, 1:2] * rot[s, 1]


def components(c0, c1):
    """Labels (index of the component's first cell) of one module's cells by
    breadth-first search over touching cells."""
    n = len(c0)
    where = {(int(c0[i]), int(c1[i])): i for i in range(n)}
    label = np.full(n, -1, np.int64)
    for i in range(n):
        if label[i] >= 0:
            continue
        label[i] = i
        queue = [i]
        while queue:
            j = queue.pop()
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    k = where.get((int(c0[j]) + dx, int(c1[j]) + dy))
                    if k is not None and label[k] < 0:
                        label[k] = i
                        queue.append(k)
    return label


def cluster(cells, geom, pitch):
    """Clusters of every (event, module) row of `cells` (synth.cells.Cells)
    with the module geometry `geom` (as_arrays()) and pitch [S, 2].
    Returns dict(offsets [E*S+1], loc [m,2], var [m,2], size [m],
    first [m] (global index of the cluster's first cell), label [n] (the
    cluster number of every cell), spacepoint [m,3])."""
    S = cells.n_surfaces
    rows = cells.n_events * S
    off = cells.offsets
    half = geom["half"].astype(np.float64)
    rot = geom["rot"].astype(np.float64).reshape(-1, 3, 3)
    centre = geom["center"].astype(np.float64)
    counts = np.zeros(rows, np.int64)
    loc, size, first, sp = [], [], [], []
    label = np.full(cells.n_cells, -1, np.int64)
    for r in range(rows):
        a, b = int(off[r]), int(off[r + 1])
        if a == b:
            continue
        s = r % S
        lab = components(cells.c0[a:b], cells.c1[a:b])
        roots = [i for i in range(b - a) if lab[i] == i]
        counts[r] = len(roots)
        base = len(loc)
        num = {root: base + k for k, root in enumerate(roots)}
        for i in range(b - a):
            label[a + i] = num[int(lab[i])]
        p0, p1 = float(pitch[s, 0]), float(pitch[s, 1])
        for root in roots:
            members = [i for i in range(b - a) if lab[i] == root]
            w = x = y = 0.0
            for i in members:
                q = float(cells.q[a + i])
                w += q
                x += q * (cells.c0[a + i] + 0.5)
                y += q * (cells.c1[a + i] + 0.5)
            l0, l1 = p0 * (x / w) - half[s, 0], p1 * (y / w) - half[s, 1]
            loc.append((l0, l1))
            size.append(len(members))
            first.append(a + root)
            sp.append(centre[s] + l0 * rot[s, 0] + l1 * rot[s, 1])
    offsets = np.zeros(rows + 1, np.int64)
    offsets[1:] = np.cumsum(counts)
    loc = np.array(loc, np.float64).reshape(-1, 2)
    var = (np.asarray(pitch, np.float64) ** 2 / 12.0)[np.repeat(np.arange(rows) % S, counts)]
    return dict(offsets=offsets, loc=loc, var=var.reshape(-1, 2), size=np.array(size, np.int64),
                first=np.array(first, np.int64), label=label, spacepoint=np.array(sp).reshape(-1, 3))
