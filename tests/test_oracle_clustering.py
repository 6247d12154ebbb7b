"""Pins of the oracle's cell clustering and measurement formation (paper
section 2: connected component analysis of the activated cells, weighted
centroids as measurements, spacepoints in global coordinates): the
partition against scipy's image labelling, centroids of hand-built clusters,
and the measurements against the simulation's truth."""
import math

import numpy as np

from synth import make_event
from synth.cells import Cells, cell_grid, make_cells


def test_components_equal_library_labelling(det_dense):
    """Every module of a mu = 20 event: the breadth-first components are the
    partition scipy.ndimage.label finds with the 3 x 3 structuring element."""
    import scipy.ndimage as nd
    from oracle import clustering as OC
    n, _ = cell_grid(det_dense)
    ev = make_event(det_dense, 6000, mu=20)
    c = make_cells(det_dense, ev, 1)
    checked = 0
    for s in range(c.n_surfaces):
        a, b = c.offsets[s], c.offsets[s + 1]
        if b - a < 2:
            continue
        grid = np.zeros((n[s, 1], n[s, 0]), np.int64)
        grid[c.c1[a:b], c.c0[a:b]] = 1
        lab, k = nd.label(grid, structure=np.ones((3, 3)))
        ref = lab[c.c1[a:b], c.c0[a:b]]
        mine = OC.components(c.c0[a:b], c.c1[a:b])
        assert len(np.unique(mine)) == k
        pairs = np.unique(np.stack([mine, ref], 1), axis=0)
        assert len(pairs) == k  # a bijection between the two labellings
        checked += 1
    assert checked > 1000


def _one_module(cells, q):
    c0 = np.array([x for x, _ in cells], np.int32)
    c1 = np.array([y for _, y in cells], np.int32)
    o = np.lexsort((c0, c1))
    return Cells(1, 1, np.array([0, len(cells)], np.int32), c0[o], c1[o], np.asarray(q, np.float32)[o],
                 np.zeros(len(cells), np.int64))


def test_centroids_of_hand_built_clusters():
    """One module, pitch (0.05, 0.2), half lengths (10, 30): a lone cell
    sits at its centre; two equal cells side by side at their midpoint;
    charges 1, 2, 1 along a row at the middle cell; an L of charges 1, 1, 2
    at the hand-computed weighted mean; a diagonal pair is one cluster; the
    variances are pitch^2 / 12."""
    from oracle import clustering as OC
    geom = dict(half=np.array([[10.0, 30.0]], np.float32), rot=np.eye(3, dtype=np.float32).reshape(1, 9),
                center=np.zeros((1, 3), np.float32))
    pitch = np.array([[0.05, 0.2]], np.float32)
    p0, p1 = float(pitch[0, 0]), float(pitch[0, 1])
    x = lambda c: (c + 0.5) * p0 - 10.0
    y = lambda c: (c + 0.5) * p1 - 30.0
    cases = [
        ([(7, 3)], [1.0], (x(7), y(3))),
        ([(7, 3), (8, 3)], [1.0, 1.0], (0.5 * (x(7) + x(8)), y(3))),
        ([(4, 9), (5, 9), (6, 9)], [1.0, 2.0, 1.0], (x(5), y(9))),
        ([(2, 2), (3, 2), (2, 3)], [1.0, 1.0, 2.0], ((x(2) * 3 + x(3)) / 4, (y(2) * 2 + y(3) * 2) / 4)),
        ([(10, 10), (11, 11)], [1.0, 3.0], ((x(10) + 3 * x(11)) / 4, (y(10) + 3 * y(11)) / 4)),
    ]
    for cells, q, want in cases:
        r = OC.cluster(_one_module(cells, q), geom, pitch)
        assert len(r["size"]) == 1 and r["size"][0] == len(cells)
        np.testing.assert_allclose(r["loc"][0], want, rtol=0, atol=1e-12)
        np.testing.assert_allclose(r["var"][0], [p0 ** 2 / 12, p1 ** 2 / 12], rtol=1e-12)
    # two clusters two columns apart stay apart, named in readout order
    r = OC.cluster(_one_module([(1, 1), (3, 1), (3, 2)], [1, 1, 1]), geom, pitch)
    assert list(r["size"]) == [1, 2] and list(r["label"]) == [0, 1, 1]


def test_measurements_against_truth(det_dense):
    """Clusters made by one particle alone on a module where it crossed
    once: the centroid lies within the cell-quantisation error of the true
    crossing (mean |residual| below a quarter pitch, none beyond a pitch and
    a half along the track's projection), and the spacepoint is on the
    module plane next to the true position."""
    from oracle import clustering as OC
    g = det_dense.as_arrays()
    n, pitch = cell_grid(det_dense)
    ev = make_event(det_dense, 6001, mu=10)
    c = make_cells(det_dense, ev, 2, noise_cells=0)
    r = OC.cluster(c, g, pitch)
    tr = ev.truth
    where = {}
    for i in range(len(tr.particle)):
        where.setdefault((int(tr.particle[i]), int(tr.surface[i])), []).append(i)
    res, dist = [], []
    rot = g["rot"].reshape(-1, 3, 3)
    for k in range(len(r["size"])):
        cell_ids = np.nonzero(r["label"] == k)[0]
        parts = np.unique(c.particle[cell_ids])
        s = int(np.searchsorted(c.offsets, cell_ids[0], side="right") - 1)
        if len(parts) != 1 or parts[0] < 0:
            continue
        hits = where.get((int(parts[0]), s), [])
        if len(hits) != 1:
            continue
        i = hits[0]
        res.append((r["loc"][k] - tr.loc[i]) / pitch[s])
        d = r["spacepoint"][k] - g["center"][s]
        assert abs(float(d @ rot[s, 2])) < 1e-4
        dist.append(np.linalg.norm(r["spacepoint"][k] - tr.pos[i]))
    res = np.array(res)
    assert len(res) > 2000
    assert np.all(np.abs(res.mean(0)) < 0.05)
    assert np.all(np.abs(res).mean(0) < 0.25) and np.abs(res).max() < 1.5
    assert np.median(dist) < 0.1


def test_spacepoints_of_truth_crossings(det_dense):
    """The spacepoint definition on the simulator's truth: the local position
    of every crossing, taken to global coordinates, is the crossing point
    the simulator computed on the helix (planes of flat modules), to the
    rounding of the FP32 module geometry (centres up to ~1.5 m: a float32
    ulp there is 1.2e-4 mm)."""
    from oracle import clustering as OC
    ev = make_event(det_dense, 6002, mu=5)
    tr = ev.truth
    sp = OC.spacepoints(det_dense.as_arrays(), tr.surface, tr.loc)
    d = np.linalg.norm(sp - tr.pos, axis=1)
    assert len(d) > 1000 and d.max() < 1.2e-4
