"""Pins of the oracle's propagation (paper section 2: RKN4 propagation of the
track parameters and their covariances) against closed forms, independent
root finding and finite differences."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

KAPPA = 2.99792458e-4


def helix_exact(p0, T0, qop, B, s):
    """Exact solution of dr/ds = T, dT/ds = kappa*qop*(T x B) for uniform B,
    written independently of the oracle (rotation about B)."""
    B = np.asarray(B, float)
    bm = np.linalg.norm(B)
    if bm == 0:
        return p0 + s * T0, T0
    b = B / bm
    om = KAPPA * qop * bm
    tpar = T0 @ b
    tperp = T0 - tpar * b
    w = np.cross(T0, b)
    a = om * s
    p = p0 + tpar * s * b + (math.sin(a) / om) * tperp + ((1 - math.cos(a)) / om) * w
    T = tpar * b + math.cos(a) * tperp + math.sin(a) * w
    return p, T


def plane_crossing(p0, T0, qop, B, c, n, s_guess):
    f = lambda s: n @ (helix_exact(p0, T0, qop, B, s)[0] - c)
    lo, hi = 0.5 * s_guess, 1.5 * s_guess + 1.0
    s = brentq(f, lo, hi, xtol=1e-13, rtol=1e-15, maxiter=200)
    return s, *helix_exact(p0, T0, qop, B, s)


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def test_straight_line_is_exact(oracle_lib):
    """B = 0: every stage vanishes, the result is the line-plane crossing."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        p0 = rng.normal(0, 10, 3)
        T0 = _unit(rng.normal(0, 1, 3) + np.array([3.0, 0, 0]))
        n = _unit(np.array([1.0, 0.2, -0.1]) + rng.normal(0, 0.1, 3))
        c = p0 + 400.0 * n + rng.normal(0, 5, 3)
        s_exact = n @ (c - p0) / (n @ T0)
        res = oracle_lib.propagate_free((0, 0, 0), np.r_[p0, T0, 0.5], c, n)
        assert res is not None
        fo, path = res
        np.testing.assert_allclose(fo[:3], p0 + s_exact * T0, atol=1e-9)
        np.testing.assert_allclose(fo[3:6], T0, atol=1e-12)
        assert abs(path - s_exact) < 1e-9


@pytest.mark.parametrize("B", [(0, 0, 2.0), (0.3, -0.4, 1.7)])
def test_helix_closed_form_tight(oracle_lib, B):
    """Uniform field (axial and tilted): RKN4 at a tight tolerance reproduces
    the exact helix crossing of a plane over ~1 m to 1e-8 mm."""
    rng = np.random.default_rng(7)
    for _ in range(12):
        p0 = rng.normal(0, 1, 3)
        T0 = _unit(np.array([1.0, rng.normal(0, 0.3), rng.normal(0, 0.5)]))
        qop = rng.choice([-1, 1]) / rng.uniform(0.6, 5.0)
        n = _unit(np.array([1.0, rng.normal(0, 0.2), rng.normal(0, 0.2)]))
        c = np.array([900.0, 0, 0]) + rng.normal(0, 20, 3)
        s_lin = n @ (c - p0) / (n @ T0)
        s, pe, Te = plane_crossing(p0, T0, qop, B, c, n, s_lin)
        res = oracle_lib.propagate_free(B, np.r_[p0, T0, qop], c, n, step_tol=1e-10, land_tol=1e-10,
                                        step_max=50.0, max_rk_steps=100000)
        assert res is not None
        fo, path = res
        assert np.max(np.abs(fo[:3] - pe)) < 1e-8
        assert np.max(np.abs(fo[3:6] - Te)) < 1e-10
        assert abs(path - s) < 1e-7


def test_helix_production_tolerance(oracle_lib):
    """Default controller (step_tol 1e-2 mm on the error estimate): true
    position error below 1e-3 mm per metre for 0.5-10 GeV tracks."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(40):
        p0 = np.zeros(3)
        T0 = _unit(np.array([1.0, 0.0, rng.uniform(-1, 1)]))
        qop = rng.choice([-1, 1]) / rng.uniform(0.5, 10.0)
        n = np.array([1.0, 0.0, 0.0])
        c = np.array([rng.uniform(200, 1000), 0, 0])
        s_lin = c[0] / T0[0]
        s, pe, Te = plane_crossing(p0, T0, qop, (0, 0, 2.0), c, n, s_lin)
        fo, path = oracle_lib.propagate_free((0, 0, 2.0), np.r_[p0, T0, qop], c, n)
        worst = max(worst, np.max(np.abs(fo[:3] - pe)) / (s / 1000.0))
    assert worst < 1e-3


def _plane_geometry(n_planes=2, positions=None, tilt=0.0):
    """A few free-standing planar modules: normal ~x, u ~y, v = z."""
    xs = positions if positions is not None else np.linspace(100.0, 100.0 * n_planes, n_planes)
    n = len(xs)
    center = np.zeros((n, 3), np.float32)
    rot = np.zeros((n, 9), np.float32)
    for i, x in enumerate(xs):
        a = tilt * (i + 1)
        nn = np.array([math.cos(a), math.sin(a), 0.0])
        u = np.array([-math.sin(a), math.cos(a), 0.0])
        v = np.array([0.0, 0.0, 1.0])
        center[i] = (x, 3.0 * i, -2.0 * i)
        rot[i] = np.r_[u, v, nn]
    return dict(center=center, rot=rot, half=np.full((n, 2), 1000.0, np.float32),
                thick=np.zeros(n, np.float32), layer=np.arange(n, dtype=np.int32),
                layer_type=np.zeros(n, np.int32), layer_pos=np.asarray(xs, np.float32) - 5.0,
                layer_lo=np.full(n, -2000.0, np.float32), layer_hi=np.full(n, 2000.0, np.float32))


def test_zero_length_transport_is_identity(oracle_lib):
    """bound -> free -> bound on the same plane: parameters unchanged and
    J_fb * J_bf = I (the conversion Jacobians are inverse)."""
    geo = _plane_geometry(1, tilt=0.3)
    inp = oracle_lib.Inputs(geo, (0, 0, 2.0))
    rng = np.random.default_rng(2)
    for _ in range(10):
        p = np.array([rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(-0.5, 0.5) + 0.3,
                      rng.uniform(1.0, 2.1), rng.choice([-1, 1]) * rng.uniform(0.1, 2)])
        cov = oracle_lib.pack_cov(np.diag([0.01, 0.02, 1e-4, 2e-4, 1e-4]))
        po, co, jac, path = oracle_lib.propagate(inp, 0, p, cov, 0)
        np.testing.assert_allclose(po, p, atol=1e-12)
        np.testing.assert_allclose(jac, np.eye(5), atol=1e-12)
        assert abs(path) < 1e-12


@pytest.mark.parametrize("B", [(0, 0, 2.0), (0.2, 0.1, 2.0), (0, 0, 0), "solenoid map"])
def test_jacobian_matches_finite_differences(oracle_lib, B):
    """The transported bound-to-bound Jacobian equals central finite
    differences of the propagate-to-plane map (tight controller); in the
    field map the position columns carry the field-gradient terms."""
    if B == "solenoid map":
        from synth.field import solenoid_map
        B = solenoid_map()
    geo = _plane_geometry(2, positions=[50.0, 450.0], tilt=0.2)
    inp = oracle_lib.Inputs(geo, B)
    tight = dict(step_tol=1e-11, land_tol=1e-12, step_max=20.0, max_rk_steps=100000)
    p = np.array([1.0, -2.0, 0.25, 1.3, 0.8])
    cov = oracle_lib.pack_cov(np.eye(5) * 1e-4)
    po, co, J, _ = oracle_lib.propagate(inp, 0, p, cov, 1, **tight)
    scale = np.array([1e-3, 1e-3, 1e-6, 1e-6, 1e-6])
    Jfd = np.zeros((5, 5))
    for j in range(5):
        d = np.zeros(5)
        d[j] = scale[j]
        a = oracle_lib.propagate(inp, 0, p + d, cov, 1, **tight)[0]
        b = oracle_lib.propagate(inp, 0, p - d, cov, 1, **tight)[0]
        Jfd[:, j] = (a - b) / (2 * scale[j])
    err = np.abs(J - Jfd) / (np.abs(Jfd) + np.abs(Jfd).max(axis=1, keepdims=True) * 1e-3 + 1e-12)
    assert err.max() < 1e-5, (J, Jfd)
    # covariance transport is J C J^T
    np.testing.assert_allclose(oracle_lib.unpack_cov(co), J @ (np.eye(5) * 1e-4) @ J.T, rtol=1e-12, atol=1e-20)
