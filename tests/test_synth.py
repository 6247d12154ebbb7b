"""Pins of the synthetic detectors and the event simulator."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.spatial import cKDTree

from synth import make_event
from synth.detector import BARREL


def test_frames_orthonormal(det_barrel, det_dense):
    for det in (det_barrel, det_dense):
        R = det.rot.astype(np.float64)
        err = np.abs(np.einsum("nij,nkj->nik", R, R) - np.eye(3)).max()
        assert err < 1e-6
        assert np.allclose(np.cross(R[:, 0], R[:, 1]), R[:, 2], atol=1e-6)


def test_envelopes_inside_modules(det_barrel, det_dense):
    """Every point of a module lies on the far side of its layer's envelope,
    so an outward track meets the envelope first."""
    for det in (det_barrel, det_dense):
        c = det.center.astype(np.float64)
        u, v = det.rot[:, 0].astype(np.float64), det.rot[:, 1].astype(np.float64)
        h = det.half.astype(np.float64)
        for s0 in (-1, 1):
            for s1 in (-1, 1):
                p = c + s0 * h[:, :1] * u + s1 * h[:, 1:] * v
                L = det.layer
                barrel = det.layer_type[L] == BARREL
                r = np.hypot(p[:, 0], p[:, 1])
                assert np.all(r[barrel] >= det.layer_pos[L][barrel] - 1e-4)
                assert np.all(np.abs(p[~barrel, 2]) >= np.abs(det.layer_pos[L][~barrel]) - 1e-4)
                assert np.all((p[barrel, 2] >= det.layer_lo[L][barrel]) & (p[barrel, 2] <= det.layer_hi[L][barrel]))
                assert np.all((r[~barrel] >= det.layer_lo[L][~barrel]) & (r[~barrel] <= det.layer_hi[L][~barrel]))


def test_barrel_phi_coverage(det_barrel):
    """Radial rays from the axis hit at least one module of every layer."""
    det = det_barrel
    c = det.center.astype(np.float64)
    R = det.rot.astype(np.float64)
    phis = np.linspace(0, 2 * math.pi, 997, endpoint=False)
    d = np.stack([np.cos(phis), np.sin(phis), np.zeros_like(phis)], -1)  # (P, 3)
    for L in range(det.n_layers):
        idx = np.nonzero(det.layer == L)[0]
        for z in (-987.0, 3.3, 611.0):
            sel = idx[np.abs(c[idx, 2] - z) < 40]
            o = np.array([0, 0, z])
            nd = d @ R[sel, 2].T                                    # (P, M)
            t = np.einsum("mj,mj->m", R[sel, 2], c[sel] - o)[None, :] / nd
            p = o + t[..., None] * d[:, None, :]                    # (P, M, 3)
            rel = p - c[sel][None]
            l0 = np.einsum("pmj,mj->pm", rel, R[sel, 0])
            l1 = np.einsum("pmj,mj->pm", rel, R[sel, 1])
            ok = (t > 0) & (np.abs(l0) <= det.half[sel, 0]) & (np.abs(l1) <= det.half[sel, 1])
            assert ok.any(axis=1).all(), (L, z)


def _brute_force_crossings(det, p0, T0, qop, bz, smax=2500.0):
    """Every module crossing of a helix found without the simulator: sample
    the exact helix, pick modules near the path (k-d tree), bracket sign
    changes of the plane distance and refine with Brent's method."""
    kappa = 2.99792458e-4
    om = -kappa * qop * bz
    st = math.hypot(T0[0], T0[1])
    ph = math.atan2(T0[1], T0[0])

    def at(s):
        a = ph + om * s
        return np.array([p0[0] + st / om * (math.sin(a) - math.sin(ph)),
                         p0[1] - st / om * (math.cos(a) - math.cos(ph)), p0[2] + T0[2] * s])

    limit = min(smax, math.pi / abs(om))
    ss = np.arange(0.0, limit, 1.0)
    pts = np.array([at(s) for s in ss])
    tree = cKDTree(det.center.astype(np.float64))
    near = set()
    for lst in tree.query_ball_point(pts[::5], 40.0):
        near.update(lst)
    out = []
    for m in near:
        c = det.center[m].astype(np.float64)
        n = det.rot[m, 2].astype(np.float64)
        f = (pts - c) @ n
        for i in np.nonzero(np.sign(f[:-1]) != np.sign(f[1:]))[0]:
            s = brentq(lambda x: (at(x) - c) @ n, ss[i], ss[i + 1], xtol=1e-12)
            d = at(s) - c
            if abs(d @ det.rot[m, 0]) <= det.half[m, 0] and abs(d @ det.rot[m, 1]) <= det.half[m, 1]:
                out.append((s, m))
    return [m for s, m in sorted(out) if s > 1e-6]


@pytest.mark.parametrize("which", ["barrel", "dense"])
def test_simulator_crossings_match_brute_force(det_barrel, det_dense_vacuum, which):
    det = det_barrel if which == "barrel" else det_dense_vacuum
    ev = make_event(det, 3, kind="tiny" if which == "barrel" else "pileup", mu=1, material=False)
    rng = np.random.default_rng(0)
    parts = rng.choice(ev.particle_pt.size, 12, replace=False)
    for p in parts:
        th = 2 * math.atan(math.exp(-ev.particle_eta[p]))
        ph = ev.particle_phi[p]
        T0 = np.array([math.cos(ph) * math.sin(th), math.sin(ph) * math.sin(th), math.cos(th)])
        qop = ev.particle_q[p] * math.sin(th) / ev.particle_pt[p]
        ref = _brute_force_crossings(det, ev.particle_vtx[p], T0, qop, 2.0)
        got = ev.truth.surface[ev.truth.particle == p].tolist()
        assert got == ref


def test_reproducible_and_sized(det_dense):
    a = make_event(det_dense, 9, mu=20)
    b = make_event(det_dense, 9, mu=20)
    assert np.array_equal(a.loc, b.loc) and np.array_equal(a.seed_params, b.seed_params)
    assert a.n_seeds > 900
    assert 6 * a.n_seeds < a.n_meas < 12 * a.n_seeds
    assert np.all(np.diff(a.offsets) >= 0) and a.offsets[-1] == a.n_meas


def test_field_simulator_reproduces_helices(det_dense):
    """The numerical simulator (RK4 through a field function, crossings on
    cubic Hermite segments) in a uniform 2 T field gives the closed-form
    simulator's crossings: the same modules in the same order, points on the
    module planes, positions within the closed-form solution's own accuracy
    (its crossing points sit up to ~4e-5 mm off the plane at grazing
    incidence) and directions within 1e-6."""
    from synth.events import pileup_particles, simulate
    from synth.fieldsim import simulate_field
    rng = np.random.Generator(np.random.PCG64(5))
    vtx, pt, eta, phi, q = pileup_particles(rng, 10)
    theta = 2 * np.arctan(np.exp(-eta))
    mom = np.stack([pt * np.cos(phi), pt * np.sin(phi), pt / np.tan(theta)], -1)
    tr = simulate(det_dense, vtx, mom, q, 2.0, rng, material=False)
    uniform = lambda p: np.broadcast_to(np.array([0.0, 0.0, 2.0]), np.shape(p)).copy()
    c = simulate_field(det_dense, vtx, mom, q, uniform, rng, material=False)
    o = np.lexsort((c["order"], c["particle"]))
    c = {k: v[o] for k, v in c.items()}
    assert np.array_equal(c["particle"], tr.particle) and np.array_equal(c["surface"], tr.surface)
    s = c["surface"]
    n = det_dense.rot[s, 2].astype(np.float64)
    on_plane = np.abs(np.einsum("ki,ki->k", n, c["pos"] - det_dense.center[s].astype(np.float64)))
    assert on_plane.max() < 1e-9
    e = np.abs(c["pos"] - tr.pos).max(1)
    assert np.percentile(e, 99) < 5e-5 and e.max() < 1e-3
    assert np.abs(c["dir"] - tr.dir).max() < 1e-6


def test_field_map_event(det_dense):
    """Truth through the solenoid map's analytic field: particles near
    |z| = 0 see ~2 T, so their crossings are close to the uniform field's;
    forward particles see less field and curve less.  Each crossing's
    recorded direction is a unit vector and every seed sits on its module."""
    from synth.field import solenoid_field
    ev = make_event(det_dense, 31, mu=4, field=solenoid_field)
    tr = ev.truth
    assert ev.n_seeds > 150 and tr.surface.size > 1500
    assert np.allclose(np.linalg.norm(tr.dir, axis=1), 1.0, atol=1e-12)
    h = det_dense.half[tr.surface].astype(np.float64)
    assert np.all(np.abs(tr.loc) <= h + 1e-9)
