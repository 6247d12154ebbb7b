"""Pins of the oracle's Kalman-filter fit and smoothers (paper section 2: a
fit with the Rauch-Tung-Striebel smoother after the CKF; section 4: the
optimal two-filter smoother): batch least squares on straight tracks, the
smoothed pulls against the simulation's truth, the gain in resolution at the
first measurement, and the agreement of the two smoothers."""
import math

import numpy as np
import pytest

from synth import make_event
from test_oracle_kalman import _OneTrack, _parallel_planes


def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


@pytest.mark.parametrize("smoother", ["rts", "two"])
def test_smoother_equals_least_squares_straight_line(oracle_lib, smoother):
    """No field, no material: the smoothed state at every plane equals the
    batch weighted least-squares fit of all measurements plus the seed
    prior (Gauss-Newton on the analytic straight-line model), carried to
    that plane; likewise its covariance.  Near phi = 0, theta = pi/2 the
    model is linear to second order, so the two agree tightly."""
    from oracle import fit as OF
    xs = np.array([100.0, 160.0, 230.0, 310.0, 400.0, 500.0])
    geo = _parallel_planes(xs)
    rng = np.random.default_rng(18)
    sig = np.array([0.015, 0.05])

    def model(q):
        l0, l1, phi, th, _ = q
        T = np.array([math.cos(phi) * math.sin(th), math.sin(phi) * math.sin(th), math.cos(th)])
        s = (xs - xs[0]) / T[0]
        return np.stack([l0 + s * T[1], l1 + s * T[2]], -1)

    for trial in range(4):
        truth = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-0.01, 0.01),
                          math.pi / 2 + rng.uniform(-0.01, 0.01), 0.5])
        meas = model(truth) + rng.normal(size=(len(xs), 2)) * sig
        seed_sig = np.array([0.05, 0.1, 2e-4, 2e-4, 0.01])
        seed = truth + rng.normal(size=5) * seed_sig
        Cs = np.diag(seed_sig ** 2)
        ev = _OneTrack(len(xs), meas, np.tile(sig ** 2, (len(xs), 1)), seed, oracle_lib.pack_cov(Cs))
        inp = oracle_lib.Inputs(geo, (0, 0, 0), ev)
        kw = dict(material=False, material_on=0, step_tol=1e-12, land_tol=1e-12)
        r = OF.fit_track(inp, 0, seed, oracle_lib.pack_cov(Cs), np.arange(len(xs)), meas,
                         np.tile(sig ** 2, (len(xs), 1)), smoother, **kw)
        assert r is not None
        q = seed.copy()
        W = np.diag(1 / np.tile(sig ** 2, len(xs)))
        Ws = np.linalg.inv(Cs)
        for _ in range(30):
            res = (meas - model(q)).ravel()
            Jm = np.zeros((2 * len(xs), 5))
            for j in range(5):
                d = np.zeros(5)
                d[j] = 1e-7
                Jm[:, j] = ((model(q + d) - model(q - d)) / 2e-7).ravel()
            Hs = Jm.T @ W @ Jm + Ws
            dq = np.linalg.solve(Hs, Jm.T @ W @ res - Ws @ (q - seed))
            q = q + dq
            if np.abs(dq).max() < 1e-14:
                break
        Cq = np.linalg.inv(Hs)
        for k in range(len(xs)):
            Jmap = np.zeros((5, 5))
            for j in range(5):
                d = np.zeros(5)
                d[j] = 1e-7
                Jmap[:2, j] = (model(q + d)[k] - model(q - d)[k]) / 2e-7
            Jmap[2, 2] = Jmap[3, 3] = Jmap[4, 4] = 1.0
            ref = np.array([*model(q)[k], q[2], q[3], q[4]])
            Ck = Jmap @ Cq @ Jmap.T
            sk = np.sqrt(np.diag(Ck))
            assert np.max(np.abs(r["params"][k] - ref) / sk) < 2e-4, (smoother, trial, k)
            np.testing.assert_allclose(np.sqrt(np.diag(r["cov"][k])), sk, rtol=2e-4)
        # the smoothed first state is much better than the filtered one
        assert r["cov"][0][2, 2] < 0.2 * r["filt_C"][0][2, 2]


def _truth_tracks(oracle_lib, det, seeds, mu, central=0.6, limit=None):
    """Particles whose every module crossing has its measurement, with the
    event's seed for that particle: (inp, ev, seed index, surfaces, ids,
    truth params [n,5])."""
    out = []
    for rs in seeds:
        ev = make_event(det, rs, mu=mu)
        inp = oracle_lib.Inputs(det.as_arrays(), (0, 0, 2.0), ev)
        tr = ev.truth
        seed_of = {int(p): i for i, p in enumerate(ev.seed_particle)}
        for part in np.unique(tr.particle):
            sel = np.nonzero(tr.particle == part)[0]
            sel = sel[np.argsort(tr.order[sel])]
            d = tr.dir[sel]
            if abs(d[0, 2]) > central or int(part) not in seed_of or len(sel) < 6:
                continue
            surfs = tr.surface[sel]
            ids = []
            for s in surfs:
                a, b = ev.offsets[s], ev.offsets[s + 1]
                hit = np.nonzero(ev.meas_particle[a:b] == part)[0]
                ids.append(a + hit[0] if len(hit) else -1)
            ids = np.array(ids)
            if np.any(ids < 0):
                continue
            truth = np.stack([tr.loc[sel, 0], tr.loc[sel, 1], np.arctan2(d[:, 1], d[:, 0]),
                              np.arccos(np.clip(d[:, 2], -1, 1)), tr.qop[sel]], -1)
            out.append((inp, ev, seed_of[int(part)], surfs, ids, truth))
            if limit and len(out) >= limit:
                return out
    return out


def test_smoothed_pulls_and_first_measurement_gain(oracle_lib, det_dense):
    """Truth helices with Highland kicks at every crossed module, Gaussian
    hits and a consistent seed: for central tracks (|cos theta| < 0.6,
    where the linearised filter is accurate) the smoothed parameters at
    every measurement have zero-mean, unit-width pulls for both smoothers,
    and at the first measurement the smoothed angles are several times
    better than the filtered ones (the reason the paper adds the
    smoother)."""
    from oracle import fit as OF
    tracks = _truth_tracks(oracle_lib, det_dense, (21, 22), mu=10)
    assert len(tracks) > 200
    for smoother in ("rts", "two"):
        P, F0, S0 = [], [], []
        for inp, ev, s, surfs, ids, truth in tracks:
            r = OF.fit_track(inp, ev.seed_surface[s], ev.seed_params[s], ev.seed_cov[s], surfs,
                             ev.loc[ids].astype(float), ev.var[ids].astype(float), smoother)
            assert r is not None
            d = r["params"] - truth
            d[:, 2] = _wrap(d[:, 2])
            P.append(d / np.sqrt(np.diagonal(r["cov"], axis1=1, axis2=2)))
            df = r["filt_p"][0] - truth[0]
            df[2] = _wrap(df[2])
            F0.append(df)
            S0.append(d[0])
        P = np.concatenate(P)
        np.testing.assert_allclose(P.mean(0), 0.0, atol=0.08)
        np.testing.assert_allclose(P.std(0), 1.0, atol=0.06)
        rms_f, rms_s = np.sqrt(np.mean(np.square(F0), 0)), np.sqrt(np.mean(np.square(S0), 0))
        assert np.all(rms_s[2:4] < 0.35 * rms_f[2:4]), (rms_s, rms_f)


def test_two_filter_agrees_with_rts(oracle_lib, det_dense):
    """The two smoothers are different algorithms: a backward gain recursion
    over the forward pass (RTS) against an independent backward information
    filter combined with the forward one (two-filter).  On one linearised
    model they are the same estimator, so with material, in 2 T, they agree
    to rounding: parameters to 1e-7 of the smoothed sigma and covariances
    to 1e-7 relative, on every measurement of every track, and both end on
    the forward filtered state.  A dropped scattering term, a wrong sign of
    the offset a or a measurement taken at the wrong index breaks this by
    orders of magnitude."""
    from oracle import fit as OF
    tracks = _truth_tracks(oracle_lib, det_dense, (23,), mu=10, limit=120)
    for material in (True, False):
        D, R = [], []
        kw = {} if material else dict(material=False, material_on=0)
        for inp, ev, s, surfs, ids, truth in tracks:
            args = (inp, ev.seed_surface[s], ev.seed_params[s], ev.seed_cov[s], surfs, ev.loc[ids].astype(float),
                    ev.var[ids].astype(float))
            r1, r2 = OF.fit_track(*args, "rts", **kw), OF.fit_track(*args, "two", **kw)
            np.testing.assert_array_equal(r1["params"][-1], r1["filt_p"][-1])
            np.testing.assert_array_equal(r2["params"][-1], r2["filt_p"][-1])
            d = r1["params"] - r2["params"]
            d[:, 2] = _wrap(d[:, 2])
            sig = np.sqrt(np.diagonal(r1["cov"], axis1=1, axis2=2))
            D.append(np.abs(d) / sig)
            R.append(np.abs(r2["cov"] - r1["cov"]) / np.sqrt(np.einsum("ni,nj->nij", sig ** 2, sig ** 2)))
        D, R = np.concatenate(D), np.concatenate(R)
        assert D.max() < 1e-7, (material, D.max(0))
        assert R.max() < 1e-7, (material, R.max())


def test_two_filter_backward_information_ignores_forward_covariance(oracle_lib, det_dense):
    """The backward filter holds no forward information: on one forward pass
    (same linearisation), replacing every forward filtered covariance by 4x
    itself changes the smoothed states, but the backward information at each
    measurement, read back as C_s^-1 - C_f^-1, stays the same to rounding.
    (A start that copied any forward covariance would scale with it.)"""
    from oracle import fit as OF
    tracks = _truth_tracks(oracle_lib, det_dense, (24,), mu=10, limit=30)
    assert len(tracks) >= 20
    worst = 0.0
    for inp, ev, s, surfs, ids, truth in tracks:
        loc, var = ev.loc[ids].astype(float), ev.var[ids].astype(float)
        fw = OF.forward(inp, ev.seed_surface[s], ev.seed_params[s], ev.seed_cov[s], surfs, loc, var)
        Ys, Ws = [], []
        for scale in (1.0, 4.0):
            f2 = dict(fw)
            f2["filt_C"] = fw["filt_C"] * scale
            xs, Cs = OF.two_filter(inp, f2, surfs, loc, var)
            Ws.append(np.linalg.inv(Cs[:-1]))
            Ys.append(Ws[-1] - np.linalg.inv(f2["filt_C"][:-1]))
        # relative to the smoothed information (the difference of two
        # inverses cancels digits where the backward part is the smaller)
        d = np.sqrt(np.einsum("nii,njj->nij", Ws[0], Ws[0]))
        worst = max(worst, float(np.max(np.abs(Ys[0] - Ys[1]) / np.maximum(d, 1e-300))))
    assert worst < 1e-9, worst
