"""Pins of the oracle's field map: bilinear interpolation reproduces a field
linear in (r, z) exactly, its gradient equals finite differences of the
interpolant, the solenoid map stays within the bilinear interpolation
bound of the analytic field, a constant map propagates like the uniform
field, propagation in the linear map matches an independent high-order
ODE solution, and the Jacobian in the solenoid map equals central finite
differences."""
import numpy as np
import pytest

from synth.field import linear_map, solenoid_field, solenoid_map


def _points(rng, n, r_max=1100.0, z_max=2900.0):
    r = rng.uniform(1.0, r_max, n)
    ph = rng.uniform(-np.pi, np.pi, n)
    z = rng.uniform(-z_max, z_max, n)
    return np.column_stack([r * np.cos(ph), r * np.sin(ph), z])


def test_linear_field_interpolated_exactly(oracle_lib):
    m = linear_map(b0=2.0, g=-2e-4)
    rng = np.random.default_rng(1)
    p = _points(rng, 500)
    B = oracle_lib.field_eval(m, p)
    r = np.hypot(p[:, 0], p[:, 1])
    br = -0.5 * r * np.float32(-2e-4)
    want = np.column_stack([br * p[:, 0] / r, br * p[:, 1] / r, 2.0 + (-2e-4) * p[:, 2]])
    # the grid values are FP32: the interpolant is exact up to their rounding
    np.testing.assert_allclose(B, want, rtol=0, atol=5e-7)


def test_gradient_equals_finite_differences(oracle_lib):
    m = solenoid_map()
    rng = np.random.default_rng(2)
    p = _points(rng, 200)
    B, G = oracle_lib.field_eval(m, p, grad=True)
    h = 1e-4
    for j in range(3):
        d = np.zeros(3)
        d[j] = h
        Gfd = (oracle_lib.field_eval(m, p + d) - oracle_lib.field_eval(m, p - d)) / (2 * h)
        # points within h of a cell edge see the kink of the bilinear interpolant
        np.testing.assert_allclose(G[:, :, j], Gfd, rtol=0, atol=2e-7 + 1e-3 * np.abs(Gfd).max())


def test_solenoid_map_within_interpolation_bound(oracle_lib):
    """|interpolant - field| <= (dr^2 |B_rr| + dz^2 |B_zz|) / 8 for a bilinear
    interpolant; here B_z'' <= 1.5 (pi/3000)^2 * 2 T/mm^2, B_r'' similarly."""
    m = solenoid_map()
    rng = np.random.default_rng(3)
    p = _points(rng, 2000)
    B = oracle_lib.field_eval(m, p)
    A = solenoid_field(p)
    bound = 25.0 / 8 * 3.0 * (np.pi / 3000.0) ** 2 * (1 + 1200 * np.pi / 6000) + 1e-6
    assert np.abs(B - A).max() <= bound
    # and the field falls from 2 T at the centre to 0.5 T at |z| = 3 m
    c = oracle_lib.field_eval(m, [[10.0, 0.0, 0.0], [10.0, 0.0, 3000.0], [10.0, 0.0, -4000.0]])
    np.testing.assert_allclose(c[:, 2], [2.0, 0.5, 0.5], atol=1e-6)


def test_constant_map_equals_uniform_field(oracle_lib):
    from synth.field import _grid
    r, z = _grid(1200.0, 3000.0, 5.0)
    vals = np.zeros((z.size, r.size, 2), np.float32)
    vals[..., 1] = 2.0
    m = dict(map=vals, nr=r.size, nz=z.size, r0=0.0, z0=-3000.0, dr=5.0, dz=5.0)
    free = np.array([30.0, 1.0, -5.0, 0.6, 0.7, 0.2, 0.9])
    free[3:6] /= np.linalg.norm(free[3:6])
    c, n = np.array([400.0, 50.0, 100.0]), np.array([1.0, 0.1, 0.0]) / np.hypot(1.0, 0.1)
    a = oracle_lib.propagate_free((0, 0, 2.0), free, c, n)
    b = oracle_lib.propagate_free(m, free, c, n)
    np.testing.assert_allclose(b[0], a[0], rtol=0, atol=1e-12)
    assert abs(a[1] - b[1]) < 1e-12


def test_linear_map_matches_independent_ode_solution(oracle_lib):
    """RKN4 at a tight tolerance in the linear map against scipy's DOP853 on
    the analytic field (the map reproduces it exactly), stopped on a plane."""
    from scipy.integrate import solve_ivp
    g = -2e-4
    m = linear_map(b0=2.0, g=g)
    kappa = 2.99792458e-4
    qop = 1.5
    free = np.array([30.0, 2.0, 40.0, 0.8, 0.5, 0.3, qop])
    free[3:6] /= np.linalg.norm(free[3:6])
    c, n = np.array([600.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0])
    out, path = oracle_lib.propagate_free(m, free, c, n, step_tol=1e-10, land_tol=1e-12, step_max=10.0,
                                          max_rk_steps=100000)
    gf = float(np.float32(g))
    b0 = 2.0

    def field(x):
        r = np.hypot(x[0], x[1])
        br = -0.5 * r * gf
        return np.array([br * x[0] / r, br * x[1] / r, b0 + gf * x[2]])

    def rhs(s, y):
        return np.concatenate([y[3:6], kappa * qop * np.cross(y[3:6], field(y[:3]))])

    ev = lambda s, y: y[0] - 600.0
    ev.terminal = True
    sol = solve_ivp(rhs, (0, 5000), free[:6], method="DOP853", rtol=1e-12, atol=1e-12, events=ev)
    y = sol.y_events[0][0]
    np.testing.assert_allclose(out[:3], y[:3], rtol=0, atol=2e-6)
    np.testing.assert_allclose(out[3:6], y[3:6], rtol=0, atol=2e-9)
    assert abs(path - sol.t_events[0][0]) < 2e-6
