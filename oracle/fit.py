"""FP64 oracle of the Kalman-filter fit of found tracks and its smoothers.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain numpy in
float64 on top of the oracle's own propagation (RKN4 with its transport
Jacobian), gain-form Kalman update and scattering, sharing nothing with the
GPU library.

What the paper fixes (section 2): after track finding, a Kalman-filter fit
runs over each found track and a Rauch-Tung-Striebel smoother carries the
information of all its measurements back to every measurement, so that
the parameters at the first measurement (the ones vertexing needs) use the
whole track.  The paper's discussion (section 4) names the optimal (two-
filter) smoother as the more stable alternative: the smoothed state is the
weighted mean of the forward filter and a backward filter.

Readings (the paper gives no formulas for the fit):

* the fit starts from the track's seed (its surface, parameters and
  covariance) and visits only the surfaces of the track's measurements, in
  the track's order; a measurement on the seed's own surface needs no leg;
* between measurement surfaces the state is propagated with the CKF's
  stepper; the covariance is transported with the leg's bound-to-bound
  Jacobian F;
* scattering (the CKF's Highland term) is added after each update, at the
  updated state: the prediction for k+1 is F (C_k|k + Q_k) F^T;
* RTS: A_k = C_k|k F^T C_k+1|k^-1, x_k|n = x_k|k + A_k (x_k+1|n - x_k+1|k),
  C_k|n = C_k|k + A_k (C_k+1|n - C_k+1|k) A_k^T; the phi difference is
  taken modulo 2 pi;
* two-filter (Fraser and Potter's optimal smoother): a backward filter
  that holds only the measurements after k, with no information from the
  forward filter, is combined with the forward filtered state at k as the
  inverse-covariance weighted mean.  The backward filter runs in
  information form (matrix Y, vector y) on the model the forward pass
  linearised: deviations from the forward filtered states,
  d_k+1 = a_k+1 + F_k+1 (d_k + w_k) with a_k+1 = x_k+1|k - x_k+1|k+1 and
  w_k the scattering of module k (covariance Q_k, evaluated at the
  forward filtered state, as the forward prediction uses it).  It starts
  from the last measurement's information alone (Y = H^T V^-1 H), so it
  needs no prior and no reversed legs; a step back is Y <- F^T Y F,
  y <- F^T (y - Y a), then the scattering (I + Y Q)^-1 applied to both;
  each measurement adds H^T V^-1 H and H^T V^-1 (m - H x_k|k).  On one
  linearised model the two smoothers are the same estimator, so RTS and
  two-filter agree to rounding; at the last measurement both are the
  forward filtered state;
* chi2 of the fit: the sum of the forward filter's chi2 increments.
"""
from __future__ import annotations

import math

import numpy as np

from . import kf_update, pack_cov, propagate, scatter, unpack_cov

_H = np.zeros((2, 5))
_H[0, 0] = _H[1, 1] = 1.0


def _wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def _leg(inp, src, p, C, dst, **cfg):
    """(params, transported cov, F) on dst, or None if the leg fails."""
    if src == dst:
        return p.copy(), C.copy(), np.eye(5)
    r = propagate(inp, src, p, pack_cov(C), dst, **cfg)
    if r is None:
        return None
    po, co, jac, _ = r
    return po, unpack_cov(co), jac


def _scatter(inp, surface, p, C, material, **cfg):
    if not material:
        return C
    return unpack_cov(scatter(inp, surface, p, pack_cov(C), **cfg))


def forward(inp, seed_surface, seed_p, seed_cov, surfaces, loc, var, material=True, **cfg):
    """The forward filter.  Returns a dict of per-measurement arrays
    pred_p [n,5], pred_C [n,5,5], F [n,5,5] (the leg into measurement k),
    filt_p, filt_C, chi2 [n], or None when a leg fails."""
    n = len(surfaces)
    out = {k: np.zeros((n, 5)) for k in ("pred_p", "filt_p")}
    out.update({k: np.zeros((n, 5, 5)) for k in ("pred_C", "filt_C", "F")})
    out["chi2"] = np.zeros(n)
    cur, p, C = int(seed_surface), np.asarray(seed_p, np.float64), unpack_cov(seed_cov)
    for k in range(n):
        r = _leg(inp, cur, p, C, int(surfaces[k]), **cfg)
        if r is None:
            return None
        pp, Cp, F = r
        pf, cf, x2 = kf_update(pp, pack_cov(Cp), loc[k], var[k])
        Cf = unpack_cov(cf)
        out["pred_p"][k], out["pred_C"][k], out["F"][k] = pp, Cp, F
        out["filt_p"][k], out["filt_C"][k], out["chi2"][k] = pf, Cf, x2
        cur, p = int(surfaces[k]), pf
        C = _scatter(inp, cur, pf, Cf, material, **cfg)
    return out


def rts(fw):
    """Rauch-Tung-Striebel smoothing of a forward pass."""
    xp, Cp, F, xf, Cf = fw["pred_p"], fw["pred_C"], fw["F"], fw["filt_p"], fw["filt_C"]
    n = xf.shape[0]
    xs, Cs = xf.copy(), Cf.copy()
    for k in range(n - 2, -1, -1):
        A = Cf[k] @ F[k + 1].T @ np.linalg.inv(Cp[k + 1])
        d = xs[k + 1] - xp[k + 1]
        d[2] = _wrap(d[2])
        xs[k] = xf[k] + A @ d
        xs[k, 2] = _wrap(xs[k, 2])
        Cs[k] = Cf[k] + A @ (Cs[k + 1] - Cp[k + 1]) @ A.T
    return xs, Cs


def two_filter(inp, fw, surfaces, loc, var, material=True, **cfg):
    """Optimal (two-filter) smoothing: the inverse-covariance weighted mean of
    the forward filtered state at k and an independent backward filter's
    information from the measurements after k, in the deviations from the
    forward filtered states of the model the forward pass linearised."""
    xp, F, xf, Cf = fw["pred_p"], fw["F"], fw["filt_p"], fw["filt_C"]
    n = xf.shape[0]
    xs, Cs = xf.copy(), Cf.copy()

    def info(k):  # the information of measurement k about d_k
        Vi = np.diag(1.0 / np.asarray(var[k], np.float64))
        r = np.asarray(loc[k], np.float64) - _H @ xf[k]
        return _H.T @ Vi @ _H, _H.T @ Vi @ r

    Y, y = info(n - 1)
    for k in range(n - 2, -1, -1):
        # step back from k+1 to k through d_k+1 = a + F (d_k + w_k)
        a = xp[k + 1] - xf[k + 1]
        a[2] = _wrap(a[2])
        Fk = F[k + 1]
        Yu, yu = Fk.T @ Y @ Fk, Fk.T @ (y - Y @ a)
        Q = _scatter(inp, int(surfaces[k]), xf[k], np.zeros((5, 5)), material, **cfg)
        M = np.linalg.inv(np.eye(5) + Yu @ Q)
        Y, y = M @ Yu, M @ yu
        Y = 0.5 * (Y + Y.T)
        # the weighted mean with the forward filtered state (deviation 0)
        Cs[k] = np.linalg.inv(np.linalg.inv(Cf[k]) + Y)
        xs[k] = xf[k] + Cs[k] @ y
        xs[k, 2] = _wrap(xs[k, 2])
        Ym, ym = info(k)
        Y, y = Y + Ym, y + ym
    return xs, Cs


def fit_track(inp, seed_surface, seed_p, seed_cov, surfaces, loc, var, smoother="rts", material=True, **cfg):
    """Fit one track: dict(params [n,5], cov [n,5,5] smoothed at each
    measurement, filt_p, filt_C, chi2) or None."""
    fw = forward(inp, seed_surface, seed_p, seed_cov, surfaces, loc, var, material, **cfg)
    if fw is None:
        return None
    if smoother == "rts":
        sm = rts(fw)
    else:
        sm = two_filter(inp, fw, surfaces, loc, var, material, **cfg)
        if sm is None:
            return None
    return dict(params=sm[0], cov=sm[1], filt_p=fw["filt_p"], filt_C=fw["filt_C"], chi2=float(fw["chi2"].sum()))


def fit_tracks(inp, ev, offsets, meas, meas_surface, seed, smoother="rts", material=True, **cfg):
    """Fit every track of a CSR (measurement ids `meas` into the event's
    loc/var, their modules `meas_surface`, track seed indices `seed`).
    Returns params [n_meas,5], cov [n_meas,15] (smoothed, NaN for a failed
    track), chi2 [n_tracks], ok [n_tracks]."""
    nt = len(offsets) - 1
    params = np.full((len(meas), 5), np.nan)
    cov = np.full((len(meas), 15), np.nan)
    chi2 = np.zeros(nt)
    ok = np.zeros(nt, np.int32)
    for t in range(nt):
        a, b = int(offsets[t]), int(offsets[t + 1])
        ids = np.asarray(meas[a:b])
        s = int(seed[t])
        r = fit_track(inp, ev.seed_surface[s], ev.seed_params[s], ev.seed_cov[s], meas_surface[a:b],
                      ev.loc[ids].astype(np.float64), ev.var[ids].astype(np.float64), smoother, material, **cfg)
        if r is None:
            continue
        ok[t] = 1
        chi2[t] = r["chi2"]
        params[a:b] = r["params"]
        cov[a:b] = pack_cov(r["cov"])
    return params, cov, chi2, ok
