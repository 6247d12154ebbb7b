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
* two-filter: a backward filter starts at the last measurement from the
  forward estimate there, with the forward covariance there multiplied by
  BACKWARD_INFLATION (100), and runs towards the first measurement.  (An
  uninformative start leaves the angles and q/p free for the first
  backward updates, and their linearisation then goes far off the track:
  with a diagonal prior of 1e4 mm^2 and 1e2 rad^2 the two smoothers
  differed by up to thousands of sigma on central tracks; with the factor
  100 by at most 0.3 sigma.  The start still holds 1 % of the forward
  information at the last measurement, a 1 % double count there.)
  Its legs reverse the track (a particle with opposite direction and
  charge follows the same curve: phi + pi, pi - theta, -q/p), and the
  scattering of surface k is added to its prediction at k.  The smoothed
  state at k is the inverse-covariance weighted mean of the forward
  filtered state at k and the backward predicted state at k (which holds
  measurements k+1..n only); at the last measurement it is the forward
  filtered state;
* chi2 of the fit: the sum of the forward filter's chi2 increments.
"""
from __future__ import annotations

import math

import numpy as np

from . import kf_update, pack_cov, propagate, scatter, unpack_cov

# the backward filter starts from the forward filtered covariance at the last
# measurement times this factor
BACKWARD_INFLATION = 100.0
_FLIP = np.diag([1.0, 1.0, 1.0, -1.0, -1.0])


def _wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def _flip(p, C):
    """The same curve traversed backwards: (l0, l1, phi + pi, pi - theta,
    -q/p); the covariance transforms with diag(1, 1, 1, -1, -1)."""
    q = np.array([p[0], p[1], _wrap(p[2] + math.pi), math.pi - p[3], -p[4]])
    return q, _FLIP @ C @ _FLIP


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


def two_filter(inp, fw, surfaces, loc, var, material=True, inflation=BACKWARD_INFLATION, **cfg):
    """Optimal (two-filter) smoothing: weighted mean of the forward filtered
    and the backward predicted state at each measurement.  None when a
    backward leg fails."""
    xf, Cf = fw["filt_p"], fw["filt_C"]
    n = xf.shape[0]
    xs, Cs = xf.copy(), Cf.copy()
    # backward filter: prior at the last measurement, then its update there
    bp = xf[n - 1].copy()
    bC = Cf[n - 1] * inflation
    pu, cu, _ = kf_update(bp, pack_cov(bC), loc[n - 1], var[n - 1])
    bp, bC = pu, unpack_cov(cu)
    for k in range(n - 2, -1, -1):
        # reverse leg from measurement k+1 to k, then the scattering of k
        q, Q = _flip(bp, bC)
        r = _leg(inp, int(surfaces[k + 1]), q, Q, int(surfaces[k]), **cfg)
        if r is None:
            return None
        q, Q, _ = r
        bp, bC = _flip(q, Q)
        bC = _scatter(inp, int(surfaces[k]), bp, bC, material, **cfg)
        # weighted mean with the forward filtered state (phi taken near it)
        b = bp.copy()
        b[2] = xf[k, 2] + _wrap(b[2] - xf[k, 2])
        Wf, Wb = np.linalg.inv(Cf[k]), np.linalg.inv(bC)
        Cs[k] = np.linalg.inv(Wf + Wb)
        xs[k] = Cs[k] @ (Wf @ xf[k] + Wb @ b)
        xs[k, 2] = _wrap(xs[k, 2])
        pu, cu, _ = kf_update(bp, pack_cov(bC), loc[k], var[k])
        bp, bC = pu, unpack_cov(cu)
    return xs, Cs


def fit_track(inp, seed_surface, seed_p, seed_cov, surfaces, loc, var, smoother="rts", material=True,
              inflation=BACKWARD_INFLATION, **cfg):
    """Fit one track: dict(params [n,5], cov [n,5,5] smoothed at each
    measurement, filt_p, filt_C, chi2) or None."""
    fw = forward(inp, seed_surface, seed_p, seed_cov, surfaces, loc, var, material, **cfg)
    if fw is None:
        return None
    if smoother == "rts":
        sm = rts(fw)
    else:
        sm = two_filter(inp, fw, surfaces, loc, var, material, inflation, **cfg)
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
