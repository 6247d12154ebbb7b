"""Pins of the oracle's Kalman-filter pieces (paper section 2: chi2 from the
covariance and the residual; filtered parameters) against the information
(weighted-means) form, batch least squares and the Highland formula."""
import math

import numpy as np
import pytest

H = np.zeros((2, 5))
H[0, 0] = H[1, 1] = 1.0


def _spd(rng, scale):
    A = rng.normal(size=(5, 5))
    C = A @ A.T + 5 * np.eye(5)
    d = np.sqrt(np.diag(C))
    C = C / np.outer(d, d)
    s = np.asarray(scale)
    return C * np.outer(s, s)


def test_gain_form_equals_information_form(oracle_lib):
    """Gain + Joseph update equals the weighted-means form
    C+ = (C^-1 + H^T V^-1 H)^-1, x+ = C+ (C^-1 x + H^T V^-1 m); chi2 is the
    innovation quadratic form."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        C = _spd(rng, [0.3, 0.8, 0.01, 0.01, 0.02])
        x = np.array([1.0, -2.0, 0.4, 1.2, 0.5]) + rng.normal(0, 0.1, 5)
        V = np.diag(rng.uniform(1e-4, 2e-2, 2))
        m = x[:2] + rng.normal(0, 0.3, 2)
        xo, co, chi2 = oracle_lib.kf_update(x, oracle_lib.pack_cov(C), m, np.diag(V))
        Ci = np.linalg.inv(C)
        Cp = np.linalg.inv(Ci + H.T @ np.linalg.inv(V) @ H)
        xp = Cp @ (Ci @ x + H.T @ np.linalg.inv(V) @ m)
        np.testing.assert_allclose(xo, xp, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(oracle_lib.unpack_cov(co), Cp, rtol=1e-8, atol=1e-14)
        r = m - x[:2]
        assert chi2 == pytest.approx(r @ np.linalg.solve(C[:2, :2] + V, r), rel=1e-12)


def test_update_is_gaussian_conditioning(oracle_lib):
    """Exact measurement (V -> 0): the filtered loc equals the measurement and
    the other parameters follow the conditional-Gaussian regression."""
    rng = np.random.default_rng(4)
    C = _spd(rng, [0.2, 0.5, 0.01, 0.01, 0.01])
    x = np.zeros(5)
    m = np.array([0.1, -0.2])
    xo, co, _ = oracle_lib.kf_update(x, oracle_lib.pack_cov(C), m, np.array([1e-14, 1e-14]))
    A, Bm = C[2:, :2], C[:2, :2]
    np.testing.assert_allclose(xo[:2], m, atol=1e-10)
    np.testing.assert_allclose(xo[2:], A @ np.linalg.solve(Bm, m), rtol=1e-7, atol=1e-12)
    Cc = C[2:, 2:] - A @ np.linalg.solve(Bm, A.T)
    np.testing.assert_allclose(oracle_lib.unpack_cov(co)[2:, 2:], Cc, rtol=1e-6, atol=1e-14)


def test_highland_increment(oracle_lib):
    """Scattering on a module at normal incidence adds theta0^2 to Var(theta)
    and theta0^2 / sin^2(theta) to Var(phi), with the PDG Highland width."""
    geo = dict(center=np.zeros((1, 3), np.float32),
               rot=np.array([[0, 1, 0, 0, 0, 1, 1, 0, 0]], np.float32),
               half=np.full((1, 2), 100.0, np.float32), thick=np.array([0.01], np.float32),
               layer=np.zeros(1, np.int32), layer_type=np.zeros(1, np.int32),
               layer_pos=np.ones(1, np.float32), layer_lo=-np.ones(1, np.float32),
               layer_hi=np.ones(1, np.float32))
    inp = oracle_lib.Inputs(geo, (0, 0, 2.0))
    for p_gev, theta in ((1.0, math.pi / 2), (0.6, 1.2)):
        params = np.array([0.0, 0.0, 0.0, theta, 1.0 / p_gev])
        cov = oracle_lib.scatter(inp, 0, params, np.zeros(15))
        # incidence: normal is x, direction (sin theta, 0, cos theta)
        x = 0.01 / abs(math.sin(theta))
        m = 0.1056583755
        beta = p_gev / math.sqrt(p_gev ** 2 + m ** 2)
        th0 = 13.6e-3 / (beta * p_gev) * math.sqrt(x) * (1 + 0.038 * math.log(x / beta ** 2))
        C = oracle_lib.unpack_cov(cov)
        assert C[3, 3] == pytest.approx(th0 ** 2, rel=1e-6)
        assert C[2, 2] == pytest.approx(th0 ** 2 / math.sin(theta) ** 2, rel=1e-6)
        assert np.count_nonzero(C) == 2
    # the textbook value: 1 GeV (beta ~ 1), 1 % X0 -> about 1.1 mrad
    assert 1.0e-3 < 13.6e-3 * 0.1 * (1 + 0.038 * math.log(0.01)) < 1.2e-3


def _parallel_planes(xs):
    n = len(xs)
    center = np.zeros((n, 3), np.float32)
    center[:, 0] = xs
    rot = np.tile(np.array([0, 1, 0, 0, 0, 1, 1, 0, 0], np.float32), (n, 1))
    return dict(center=center, rot=rot, half=np.full((n, 2), 500.0, np.float32),
                thick=np.zeros(n, np.float32), layer=np.arange(n, dtype=np.int32),
                layer_type=np.zeros(n, np.int32), layer_pos=np.asarray(xs, np.float32) - 1.0,
                layer_lo=np.full(n, -2000.0, np.float32), layer_hi=np.full(n, 2000.0, np.float32))


class _OneTrack:
    """Single seed and one measurement per plane in the layout of synth.Event."""

    def __init__(self, n_surf, meas, var, seed_p, seed_cov):
        self.n_events, self.n_surfaces = 1, n_surf
        self.offsets = np.arange(n_surf + 1, dtype=np.int32)
        self.loc = np.asarray(meas, np.float32)
        self.var = np.asarray(var, np.float32)
        self.seed_event = np.zeros(1, np.int32)
        self.seed_surface = np.zeros(1, np.int32)
        self.seed_params = np.asarray(seed_p, np.float64)[None]
        self.seed_cov = np.asarray(seed_cov, np.float64)[None]


@pytest.mark.parametrize("spread,seed_angle_sigma,bound", [(0.01, 2e-4, 2e-5), (0.3, 2e-3, 1e-2)])
def test_filter_equals_least_squares_straight_line(oracle_lib, spread, seed_angle_sigma, bound):
    """No field, no material: the CKF's filtered state at the last measurement
    equals the batch weighted least-squares fit (seed prior + all residuals),
    solved by Gauss-Newton with an analytic straight-line model, and the
    chi2 sum equals the least-squares minimum.  The filter linearises the
    model at its running estimate, so the two differ at second order: the
    straight-line model is linear to second order at phi = 0, theta = pi/2,
    where they must agree tightly; elsewhere the difference is small."""
    xs = np.array([100.0, 160.0, 230.0, 310.0, 400.0, 500.0])
    geo = _parallel_planes(xs)
    rng = np.random.default_rng(8)
    sig = np.array([0.015, 0.05])

    def model(q):  # q = bound params on plane 0 -> local positions on all planes
        l0, l1, phi, th, _ = q
        T = np.array([math.cos(phi) * math.sin(th), math.sin(phi) * math.sin(th), math.cos(th)])
        s = (xs - xs[0]) / T[0]
        return np.stack([l0 + s * T[1], l1 + s * T[2]], -1)

    for trial in range(5):
        truth = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-spread, spread),
                          math.pi / 2 + rng.uniform(-spread, spread), 0.5])
        meas = model(truth) + rng.normal(size=(len(xs), 2)) * sig
        seed_sig = np.array([0.05, 0.1, seed_angle_sigma, seed_angle_sigma, 0.01])
        seed = truth + rng.normal(size=5) * seed_sig
        Cs = np.diag(seed_sig ** 2)
        ev = _OneTrack(len(xs), meas, np.tile(sig ** 2, (len(xs), 1)), seed, oracle_lib.pack_cov(Cs))
        inp = oracle_lib.Inputs(geo, (0, 0, 0), ev)
        out = oracle_lib.ckf_find(inp, n_threads=1, material_on=0, min_meas=len(xs), chi2_max=1e9,
                                  step_tol=1e-12, land_tol=1e-12)
        assert out["n_tracks"] == 1
        assert list(out["meas"]) == list(range(len(xs)))
        # Gauss-Newton on the 4 geometric parameters (q/p unobservable at B=0)
        q = seed.copy()
        W = np.diag(1 / np.tile(sig ** 2, len(xs)))
        Ws = np.linalg.inv(Cs)
        for _ in range(30):
            r = (meas - model(q)).ravel()
            Jm = np.zeros((2 * len(xs), 5))
            for j in range(5):
                d = np.zeros(5)
                d[j] = 1e-7
                Jm[:, j] = ((model(q + d) - model(q - d)) / 2e-7).ravel()
            Hs = Jm.T @ W @ Jm + Ws
            g = Jm.T @ W @ r - Ws @ (q - seed)
            dq = np.linalg.solve(Hs, g)
            q = q + dq
            if np.abs(dq).max() < 1e-14:
                break
        Cq = np.linalg.inv(Hs)
        chi2_min = ((meas - model(q)).ravel() ** 2 @ np.diag(W)) + (q - seed) @ Ws @ (q - seed)
        # map the fit to the last plane
        l_last = model(q)[-1]
        fit_last = np.array([l_last[0], l_last[1], q[2], q[3], q[4]])
        Jmap = np.zeros((5, 5))
        for j in range(5):
            d = np.zeros(5)
            d[j] = 1e-7
            a, b = model(q + d)[-1], model(q - d)[-1]
            Jmap[:2, j] = (a - b) / 2e-7
        Jmap[2, 2] = Jmap[3, 3] = Jmap[4, 4] = 1.0
        C_last = Jmap @ Cq @ Jmap.T
        sig_last = np.sqrt(np.diag(C_last))
        assert np.max(np.abs(out["params"][0] - fit_last) / sig_last) < bound
        Co = oracle_lib.unpack_cov(out["cov"][0])
        np.testing.assert_allclose(np.sqrt(np.diag(Co)), sig_last, rtol=bound)
        assert out["chi2"][0] == pytest.approx(chi2_min, rel=bound, abs=1e-6)
