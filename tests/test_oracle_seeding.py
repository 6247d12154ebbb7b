"""Pins of the oracle's triplet seeding and helix parameter estimation
(paper section 2): the circle through three points, parameters of exact
helices, the cut definitions on hand-placed points, and seeding efficiency
and purity on clusters of simulated events."""
import math

import numpy as np
import pytest

from synth import make_event
from synth.cells import cell_grid, make_cells


def test_circle_through_three_points():
    from oracle import seeding as OS
    rng = np.random.default_rng(3)
    for _ in range(200):
        cx, cy, R = rng.uniform(-500, 500), rng.uniform(-500, 500), rng.uniform(50, 5000)
        a = np.sort(rng.uniform(0, 2 * math.pi, 3))
        pts = [(cx + R * math.cos(t), cy + R * math.sin(t)) for t in a]
        ux, uy, r = OS.circle(*pts[0], *pts[1], *pts[2])
        assert abs(ux - cx) < 1e-7 * R and abs(uy - cy) < 1e-7 * R and abs(r - R) < 1e-7 * R
    assert OS.circle(0, 0, 1, 1, 2, 2)[2] == math.inf


@pytest.mark.parametrize("q", [1.0, -1.0])
def test_estimate_on_exact_helices(q):
    """Three points of a helix from the beam line in a 2 T field (kappa
    q/p (T x B) for the turning): the estimate gives back phi at the first
    point, theta and q/p."""
    from oracle import seeding as OS
    rng = np.random.default_rng(4 if q > 0 else 5)
    bz = 2.0
    for _ in range(100):
        pt, phi0 = rng.uniform(0.5, 20.0), rng.uniform(-math.pi, math.pi)
        theta = rng.uniform(0.5, 2.6)
        R = pt / (OS.KAPPA * bz)
        # transverse motion: the direction turns by -q s / R (clockwise for q > 0 when Bz > 0)
        def point(s):
            a = phi0 - q * s / R
            x = q * R * (math.sin(phi0) - math.sin(a))   # integral of cos(phi0 - q s'/R)
            y = q * R * (math.cos(a) - math.cos(phi0))   # integral of sin(phi0 - q s'/R)
            return np.array([x, y, s / math.tan(theta)]), a
        pB, aB = point(30.0)
        pM, _ = point(70.0)
        pT, _ = point(120.0)
        phi, th, qop = OS.estimate(pB, pM, pT, bz)
        assert abs(((phi - aB) + math.pi) % (2 * math.pi) - math.pi) < 1e-9
        assert abs(th - theta) < 1e-9
        assert qop == pytest.approx(q * math.sin(theta) / pt, rel=1e-9)


def test_cuts_on_hand_placed_points():
    """Three points on a straight radial line from the origin pass (d0 = 0,
    infinite radius); moving the middle sideways by 3 mm fails the d0 cut;
    a 0.15 rad azimuth step fails the doublet cut; cot 3.2 fails the cot
    cut; a top one layer below the middle is no triplet."""
    from oracle import seeding as OS
    phi = 0.3
    pts = lambda r, z, dphi=0.0: [r * math.cos(phi + dphi), r * math.sin(phi + dphi), z]
    xyz = np.array([pts(30, 3), pts(70, 7), pts(120, 12)])
    assert [t[:3] for t in OS.triplets(xyz, [0, 1, 2], 2.0)] == [(1, 0, 2)]
    side = xyz.copy()
    side[1, :2] += 3.0 * np.array([-math.sin(phi), math.cos(phi)])
    assert OS.triplets(side, [0, 1, 2], 2.0) == []
    assert OS.triplets(np.array([pts(30, 3), pts(70, 7, 0.15), pts(120, 12, 0.15)]), [0, 1, 2], 2.0) == []
    assert OS.triplets(np.array([pts(30, 96), pts(70, 224), pts(120, 384)]), [0, 1, 2], 2.0) == []
    assert OS.triplets(xyz, [0, 2, 1], 2.0) == []


def test_seeding_on_clusters(det_dense):
    """Clusters of a mu = 20 event on the four pixel barrel layers: over 90 %
    of the seeds have three clusters of one particle, the charge is always
    right on those, their parameters match the truth at the bottom crossing
    within the seeds' stated widths, and every central particle (|eta| <
    1.2, pT > 0.6 GeV, |z_vertex| < 150 mm) gets a seed."""
    from oracle import clustering as OC, seeding as OS
    g = det_dense.as_arrays()
    _, pitch = cell_grid(det_dense)
    ev = make_event(det_dense, 6000, mu=20)
    c = make_cells(det_dense, ev, 1)
    r = OC.cluster(c, g, pitch)
    rows = np.repeat(np.arange(c.n_surfaces), np.diff(r["offsets"]))
    layer = g["layer"][rows]
    li = np.where(layer < 4, layer, -1)
    sd = OS.seeds(r["spacepoint"].astype(np.float32).astype(np.float64), li, rows,
                  r["loc"].astype(np.float32).astype(np.float64), 2.0)
    lab = r["label"]
    o = np.lexsort((-c.q, lab))
    first = o[np.r_[True, lab[o][1:] != lab[o][:-1]]]
    cp = np.full(len(rows), -1)
    cp[lab[first]] = c.particle[first]
    pure = (cp[sd["bottom"]] == cp[sd["middle"]]) & (cp[sd["middle"]] == cp[sd["top"]]) & (cp[sd["bottom"]] >= 0)
    assert len(pure) > 1000 and pure.mean() > 0.9
    tr = ev.truth
    key = {(int(tr.particle[i]), int(tr.surface[i])): i for i in range(len(tr.particle))}
    pulls = []
    for k in np.nonzero(pure)[0]:
        i = key[(int(cp[sd["bottom"][k]]), int(sd["surface"][k]))]
        d = tr.dir[i]
        t = np.array([tr.loc[i, 0], tr.loc[i, 1], math.atan2(d[1], d[0]), math.acos(d[2]), tr.qop[i]])
        e = sd["params"][k] - t
        e[2] = (e[2] + math.pi) % (2 * math.pi) - math.pi
        assert np.sign(sd["params"][k][4]) == np.sign(t[4])
        pulls.append(e / np.sqrt(sd["cov"][k][[0, 5, 9, 12, 14]]))
    P = np.abs(np.array(pulls))
    assert np.all(np.percentile(P, 95, axis=0) < 3.0)
    seeded = set(cp[sd["bottom"][pure]])
    cen = [p for p in range(len(ev.particle_pt))
           if abs(ev.particle_eta[p]) < 1.2 and ev.particle_pt[p] > 0.6 and abs(ev.particle_vtx[p, 2]) < 150]
    assert len(cen) > 200 and all(p in seeded for p in cen)
