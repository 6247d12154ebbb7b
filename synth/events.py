"""Seeded synthetic events: particles, truth trajectories, measurements, seeds.

The paper's workloads are Geant4 ttbar events with pileup in the Open Data
Detector (section 3), which are not available.  These events stand in for
them with the multiplicities and distributions of the named configurations:

* ``tiny``: 100 muons from the origin (vertex sigma 0.01 mm), pT uniform
  1-10 GeV, eta uniform [-1, 1].
* ``pileup``: 50 * mu charged muons (mu = 200 gives 10k), vertex sigma (0.01,
  0.01, 50) mm, pT from a pT^-3 spectrum on [0.5, 100] GeV, eta uniform
  [-2.5, 2.5].

Truth trajectories are exact helices in a uniform axial field (closed-form
crossings with the barrel planes, the disk planes and the layer envelopes),
or integrated numerically through a given field (synth.fieldsim), kinked at every crossed module by a Gaussian multiple-scattering kick of the
Highland width when the module has material.  Each crossing yields a hit with
probability ``eff``, smeared by the module's resolution; each module also
carries one uniform noise hit with probability ``noise``.  Seeds are the true
bound parameters at the particle's first crossing, smeared by fixed widths
(0.2 mm, 0.6 mm, 10 mrad, 10 mrad, 1 % of |q/p|) with the matching diagonal
covariance.

This module is a simulator: it holds no propagation, search or fitting
arithmetic of the track finder.  Random draws use numpy's PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .detector import BARREL, DISK, Detector

C_LIGHT = 2.99792458e-4        # GeV / (T mm) per unit charge
MUON_MASS = 0.1056583755       # GeV
SEED_SIGMA = (0.2, 0.6, 0.01, 0.01, 0.01)  # loc0, loc1, phi, theta, rel. q/p
EPS_PATH = 1e-6                # mm: crossings closer than this are "here"


# --------------------------------------------------------------------------
# particles

def tiny_particles(rng, n=100):
    vtx = rng.normal(0.0, 0.01, size=(n, 3))
    pt = rng.uniform(1.0, 10.0, n)
    eta = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(-math.pi, math.pi, n)
    q = rng.choice([-1.0, 1.0], n)
    return vtx, pt, eta, phi, q


def pileup_particles(rng, mu):
    n = int(round(50 * mu))
    vtx = np.stack([rng.normal(0.0, 0.01, n), rng.normal(0.0, 0.01, n),
                    rng.normal(0.0, 50.0, n)], -1)
    u = rng.uniform((0.5 / 100.0) ** 2, 1.0, n)
    pt = 0.5 / np.sqrt(u)
    eta = rng.uniform(-2.5, 2.5, n)
    phi = rng.uniform(-math.pi, math.pi, n)
    q = rng.choice([-1.0, 1.0], n)
    return vtx, pt, eta, phi, q


# --------------------------------------------------------------------------
# closed-form helix pieces (uniform field along z, Bz != 0)

class _Helix:
    """Helix of a set of particles: transverse circle centre (xc, yc), signed
    turning rate om (rad per mm of path), transverse speed st, start angle."""

    def __init__(self, pos, T, qop, bz):
        self.pos, self.T = pos, T
        self.om = -C_LIGHT * qop * bz
        self.st = np.hypot(T[:, 0], T[:, 1])
        self.phi0 = np.arctan2(T[:, 1], T[:, 0])
        self.xc = pos[:, 0] - self.st * np.sin(self.phi0) / self.om
        self.yc = pos[:, 1] + self.st * np.cos(self.phi0) / self.om

    def sel(self, i):
        h = _Helix.__new__(_Helix)
        for k in ("pos", "T", "om", "st", "phi0", "xc", "yc"):
            setattr(h, k, getattr(self, k)[i])
        return h

    def at(self, s):
        """Position and direction after path s (broadcast over trailing dims)."""
        om, st = self.om, self.st
        if s.ndim == 2:
            om, st = om[:, None], st[:, None]
            phi0, xc, yc = self.phi0[:, None], self.xc[:, None], self.yc[:, None]
            z0, tz = self.pos[:, 2][:, None], self.T[:, 2][:, None]
        else:
            phi0, xc, yc, z0, tz = self.phi0, self.xc, self.yc, self.pos[:, 2], self.T[:, 2]
        psi = phi0 + om * s
        p = np.stack([xc + st * np.sin(psi) / om, yc - st * np.cos(psi) / om,
                      z0 + tz * s], -1)
        d = np.stack([st * np.cos(psi), st * np.sin(psi), np.broadcast_to(tz, psi.shape)], -1)
        return p, d

    def path_to_angle(self, psi):
        """Smallest path > EPS_PATH reaching circle angle psi (inf if none)."""
        om = self.om if psi.ndim == 1 else self.om[:, None]
        phi0 = self.phi0 if psi.ndim == 1 else self.phi0[:, None]
        sg = np.sign(om)
        dpsi = np.mod((psi - phi0) * sg, 2.0 * math.pi)
        s = dpsi / np.abs(om)
        return np.where(s > EPS_PATH, s, s + 2.0 * math.pi / np.abs(om))

    def cross_cylinder(self, R):
        """Smallest positive path to r = R (inf if the circle misses it)."""
        d = np.maximum(np.hypot(self.xc, self.yc), 1e-300)
        rho = self.st / np.abs(self.om)
        a = (R * R - rho * rho + d * d) / (2.0 * d)
        h2 = R * R - a * a
        ok = h2 >= 0.0
        h = np.sqrt(np.where(ok, h2, 0.0))
        ex, ey = self.xc / d, self.yc / d
        best = np.full(self.om.shape, np.inf)
        for sgn in (1.0, -1.0):
            px = a * ex - sgn * h * ey
            py = a * ey + sgn * h * ex
            sps = (px - self.xc) * self.om / self.st
            cps = -(py - self.yc) * self.om / self.st
            s = self.path_to_angle(np.arctan2(sps, cps))
            best = np.minimum(best, np.where(ok, s, np.inf))
        return best

    def cross_zplane(self, z):
        tz = self.T[:, 2] if np.ndim(z) == 0 else self.T[:, 2][:, None]
        z0 = self.pos[:, 2] if np.ndim(z) == 0 else self.pos[:, 2][:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (z - z0) / tz
        return np.where(np.isfinite(s) & (s > EPS_PATH), s, np.inf)

    def cross_axial_plane(self, nx, ny, dist):
        """Smallest positive path to the plane nx x + ny y = dist (a plane
        containing the z direction).  nx, ny, dist have shape (M, k)."""
        om, st = self.om[:, None], self.st[:, None]
        g = (dist - nx * self.xc[:, None] - ny * self.yc[:, None]) * om / st
        ok = np.abs(g) <= 1.0
        a = np.arcsin(np.clip(g, -1.0, 1.0))
        phin = np.arctan2(ny, nx)
        s1 = self.path_to_angle(phin + a)
        s2 = self.path_to_angle(phin + math.pi - a)
        return np.where(ok, np.minimum(s1, s2), np.inf)


# --------------------------------------------------------------------------
# truth simulation

def _lattice_candidates(det: Detector, L: int, p):
    """Module ids of layer L in the 3x3 lattice neighbourhood of points p
    (M, 3): every module a trajectory can cross near p.  Returns (M, 9)."""
    lat = det.lattice[L]
    phi = np.arctan2(p[:, 1], p[:, 0])
    if lat["type"] == BARREL:
        nphi, nz = lat["nphi"], lat["nz"]
        i0 = np.floor(np.mod(phi, 2 * math.pi) * nphi / (2 * math.pi)).astype(np.int64)
        j0 = np.rint((p[:, 2] - lat["z0"]) / lat["pitch"]).astype(np.int64)
        out = []
        for dj in (-1, 0, 1):
            j = np.clip(j0 + dj, 0, nz - 1)
            for di in (-1, 0, 1):
                i = np.mod(i0 + di, nphi)
                out.append(lat["base"] + j * nphi + i)
        return np.stack(out, -1)
    out = []
    for ring in lat["rings"]:
        nphi = ring["nphi"]
        i0 = np.floor(np.mod(phi, 2 * math.pi) * nphi / (2 * math.pi)).astype(np.int64)
        for di in (-1, 0, 1):
            out.append(ring["base"] + np.mod(i0 + di, nphi))
    return np.stack(out, -1)


def _module_crossings(det, hel: _Helix, cand):
    """Exact crossings of the helices with candidate modules (M, k): path
    (inf where the module is missed), local coordinates."""
    c = det.center[cand].astype(np.float64)
    R = det.rot[cand].astype(np.float64)
    n = R[..., 2, :]
    barrel = det.layer_type[det.layer[cand]] == BARREL
    s_b = hel.cross_axial_plane(n[..., 0], n[..., 1], np.einsum("mki,mki->mk", n, c))
    s_d = hel.cross_zplane(c[..., 2])
    s = np.where(barrel, s_b, s_d)
    sf = np.where(np.isfinite(s), s, 0.0)
    p, _ = hel.at(sf)
    d = p - c
    l0 = np.einsum("mki,mki->mk", R[..., 0, :], d)
    l1 = np.einsum("mki,mki->mk", R[..., 1, :], d)
    h = det.half[cand].astype(np.float64)
    inside = (np.abs(l0) <= h[..., 0]) & (np.abs(l1) <= h[..., 1])
    return np.where(inside & np.isfinite(s), s, np.inf), l0, l1


def _layer_envelopes(det, hel: _Helix):
    """(M, L) path to each layer's envelope within its extent (inf if none)."""
    M, Ln = hel.om.shape[0], det.n_layers
    S = np.full((M, Ln), np.inf)
    for L in range(Ln):
        pos, lo, hi = float(det.layer_pos[L]), float(det.layer_lo[L]), float(det.layer_hi[L])
        if det.layer_type[L] == BARREL:
            s = hel.cross_cylinder(pos)
            sf = np.where(np.isfinite(s), s, 0.0)
            z = hel.pos[:, 2] + hel.T[:, 2] * sf
            ok = np.isfinite(s) & (z >= lo) & (z <= hi)
        else:
            s = hel.cross_zplane(pos)
            sf = np.where(np.isfinite(s), s, 0.0)
            p, _ = hel.at(sf)
            r = np.hypot(p[:, 0], p[:, 1])
            ok = np.isfinite(s) & (r >= lo) & (r <= hi)
        S[:, L] = np.where(ok, s, np.inf)
    return S


def highland(p, mass, x):
    """Highland width of the plane scattering angle for a unit charge."""
    beta = p / np.sqrt(p * p + mass * mass)
    return 0.0136 / (beta * p) * np.sqrt(x) * (1.0 + 0.038 * np.log(x / (beta * beta)))


@dataclass
class Truth:
    """Ordered module crossings of every particle (pre-kick state)."""
    particle: np.ndarray   # (k,) int64
    surface: np.ndarray    # (k,) int64
    loc: np.ndarray        # (k, 2)
    pos: np.ndarray        # (k, 3)
    dir: np.ndarray        # (k, 3)
    qop: np.ndarray        # (k,)
    order: np.ndarray      # (k,) crossing index along the particle


def simulate(det: Detector, vtx, mom, q, bz, rng, material=True, max_cross=80) -> Truth:
    N = vtx.shape[0]
    pos = vtx.astype(np.float64).copy()
    p = np.linalg.norm(mom, axis=1)
    T = mom / p[:, None]
    qop = q / p
    cur = np.full(N, -1, np.int64)
    turned = np.zeros(N)
    count = np.zeros(N, np.int64)
    alive = np.ones(N, bool)
    rec = {k: [] for k in ("particle", "surface", "loc", "pos", "dir", "qop", "order")}
    for _ in range(4 * max_cross):
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        hel = _Helix(pos[idx], T[idx], qop[idx], bz)
        limit = (math.pi - turned[idx]) / np.abs(hel.om)     # first half turn only
        S = _layer_envelopes(det, hel)
        S = np.where(S < limit[:, None], S, np.inf)
        order = np.argsort(S, axis=1)[:, :2]
        cands, paths, locs = [], [], []
        # modules near the two nearest layer envelope crossings
        for slot in range(2):
            Ls = order[:, slot]
            sL = S[np.arange(idx.size), Ls]
            cm = np.full((idx.size, 9), -1, np.int64)
            for L in np.unique(Ls[np.isfinite(sL)]):
                m = np.nonzero((Ls == L) & np.isfinite(sL))[0]
                pe, _ = hel.sel(m).at(sL[m])
                cm[m] = _lattice_candidates(det, int(L), pe)
            cands.append(cm)
        # overlapping neighbours of the current module
        on = np.nonzero(cur[idx] >= 0)[0]
        cm = np.full((idx.size, 9), -1, np.int64)
        if on.size:
            for L in np.unique(det.layer[cur[idx[on]]]):
                m = on[det.layer[cur[idx[on]]] == L]
                cm[m] = _lattice_candidates(det, int(L), pos[idx[m]])
        cands.append(cm)
        cand = np.concatenate(cands, axis=1)
        valid = (cand >= 0) & (cand != cur[idx][:, None])
        cs = np.where(valid, cand, 0)
        s, l0, l1 = _module_crossings(det, hel, cs)
        s = np.where(valid & (s < limit[:, None]), s, np.inf)
        k = np.argmin(s, axis=1)
        sbest = s[np.arange(idx.size), k]
        hit = np.isfinite(sbest)
        # particles with no module crossing: skip past the two layers, or exit
        nohit = ~hit
        far = np.where(np.isfinite(S[np.arange(idx.size), order[:, 1]]),
                       S[np.arange(idx.size), order[:, 1]],
                       S[np.arange(idx.size), order[:, 0]])
        move = nohit & np.isfinite(far)
        if move.any():
            m = np.nonzero(move)[0]
            pe, de = hel.sel(m).at(far[m])
            pos[idx[m]], T[idx[m]] = pe, de
            turned[idx[m]] += far[m] * np.abs(hel.om[m])
            cur[idx[m]] = -1
        alive[idx[nohit & ~move]] = False
        if not hit.any():
            continue
        m = np.nonzero(hit)[0]
        gi = idx[m]
        surf = cs[m, k[m]]
        pe, de = hel.sel(m).at(sbest[m])
        rec["particle"].append(gi)
        rec["surface"].append(surf)
        rec["loc"].append(np.stack([l0[m, k[m]], l1[m, k[m]]], -1))
        rec["pos"].append(pe)
        rec["dir"].append(de)
        rec["qop"].append(qop[gi])
        rec["order"].append(count[gi].copy())
        count[gi] += 1
        turned[gi] += sbest[m] * np.abs(hel.om[m])
        pos[gi], cur[gi] = pe, surf
        if material:
            t = det.thick[surf].astype(np.float64)
            nrm = det.rot[surf, 2].astype(np.float64)
            cosa = np.abs(np.einsum("ki,ki->k", nrm, de))
            x = t / np.maximum(cosa, 1e-12)
            th0 = np.where(t > 0, highland(1.0 / np.abs(qop[gi]), MUON_MASS, np.maximum(x, 1e-30)), 0.0)
            theta = np.arccos(np.clip(de[:, 2], -1.0, 1.0)) + th0 * rng.standard_normal(gi.size)
            phi = np.arctan2(de[:, 1], de[:, 0]) + th0 * rng.standard_normal(gi.size) / np.sin(
                np.arccos(np.clip(de[:, 2], -1.0, 1.0)))
            de = np.stack([np.cos(phi) * np.sin(theta), np.sin(phi) * np.sin(theta), np.cos(theta)], -1)
        T[gi] = de
        alive[gi[count[gi] >= max_cross]] = False
    cat = {k: (np.concatenate(v) if v else np.zeros((0,) + ((2,) if k == "loc" else (3,) if k in ("pos", "dir") else ())))
           for k, v in rec.items()}
    o = np.lexsort((cat["order"], cat["particle"]))
    return Truth(**{k: v[o] for k, v in cat.items()})


# --------------------------------------------------------------------------
# events

@dataclass
class Event:
    """One or more events in the layout the track finders take.

    Measurements are grouped by (event, surface): those of event e on surface
    s are rows ``offsets[e*S + s] : offsets[e*S + s + 1]``; a measurement's id
    is its row.  Seeds carry their event index."""
    n_events: int
    n_surfaces: int
    offsets: np.ndarray     # (E*S + 1,) int32
    loc: np.ndarray         # (n, 2) float32
    var: np.ndarray         # (n, 2) float32
    meas_particle: np.ndarray  # (n,) int64 global particle index, -1 noise
    seed_event: np.ndarray  # (k,) int32
    seed_surface: np.ndarray  # (k,) int32
    seed_params: np.ndarray   # (k, 5) float64  loc0 loc1 phi theta q/p
    seed_cov: np.ndarray      # (k, 15) float64 packed upper triangle
    seed_particle: np.ndarray  # (k,) int64
    seed_truth: np.ndarray    # (k, 5) unsmeared parameters
    particle_pt: np.ndarray
    particle_eta: np.ndarray
    particle_phi: np.ndarray
    particle_q: np.ndarray
    particle_vtx: np.ndarray
    particle_nhits: np.ndarray
    particle_event: np.ndarray
    truth: Truth

    @property
    def n_meas(self):
        return int(self.loc.shape[0])

    @property
    def n_seeds(self):
        return int(self.seed_params.shape[0])


def _pack_diag(sig):
    cov = np.zeros((sig.shape[0], 15))
    for i, k in enumerate((0, 5, 9, 12, 14)):
        cov[:, k] = sig[:, i] ** 2
    return cov


def make_event(det: Detector, rng_seed: int, kind="pileup", mu=200.0, bz=2.0,
               eff=0.99, noise=0.01, material=None, smear_seeds=True, field=None) -> Event:
    """One event.  The truth follows closed-form helices in the uniform axial
    field bz, or, with ``field`` (a function of points [M, 3] in mm giving
    the field [M, 3] in tesla, e.g. synth.field.solenoid_field), is
    integrated numerically through that field (synth.fieldsim)."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    if kind == "tiny":
        vtx, pt, eta, phi, q = tiny_particles(rng)
    else:
        vtx, pt, eta, phi, q = pileup_particles(rng, mu)
    if material is None:
        material = bool(np.any(det.thick > 0))
    theta = 2.0 * np.arctan(np.exp(-eta))
    mom = np.stack([pt * np.cos(phi), pt * np.sin(phi), pt / np.tan(theta)], -1)
    if field is None:
        tr = simulate(det, vtx, mom, q, bz, rng, material=material)
    else:
        from .fieldsim import simulate_field
        cat = simulate_field(det, vtx, mom, q, field, rng, material=material)
        o = np.lexsort((cat["order"], cat["particle"]))
        tr = Truth(**{k: v[o] for k, v in cat.items()})
    S = det.n_surfaces
    sig = det.sigma().astype(np.float64)
    # signal hits
    keep = rng.uniform(size=tr.surface.size) < eff
    hs = tr.surface[keep]
    hloc = tr.loc[keep] + rng.standard_normal((hs.size, 2)) * sig[hs]
    hpart = tr.particle[keep]
    # noise hits
    ns = np.nonzero(rng.uniform(size=S) < noise)[0]
    nloc = (rng.uniform(-1.0, 1.0, size=(ns.size, 2)) * det.half[ns].astype(np.float64))
    surf = np.concatenate([hs, ns])
    loc = np.concatenate([hloc, nloc])
    part = np.concatenate([hpart, np.full(ns.size, -1)])
    o = np.argsort(surf, kind="stable")
    surf, loc, part = surf[o], loc[o], part[o]
    offsets = np.zeros(S + 1, np.int64)
    np.add.at(offsets, surf + 1, 1)
    offsets = np.cumsum(offsets)
    var = sig[surf] ** 2
    # seeds: first crossing of every particle that crossed something
    first = np.nonzero(tr.order == 0)[0]
    sp = tr.particle[first]
    d = tr.dir[first]
    truth5 = np.stack([tr.loc[first, 0], tr.loc[first, 1], np.arctan2(d[:, 1], d[:, 0]),
                       np.arccos(np.clip(d[:, 2], -1, 1)), tr.qop[first]], -1)
    sig5 = np.stack([np.full(sp.size, SEED_SIGMA[0]), np.full(sp.size, SEED_SIGMA[1]),
                     np.full(sp.size, SEED_SIGMA[2]), np.full(sp.size, SEED_SIGMA[3]),
                     SEED_SIGMA[4] * np.abs(tr.qop[first])], -1)
    params = truth5 + (rng.standard_normal(truth5.shape) * sig5 if smear_seeds else 0.0)
    nh = np.bincount(hpart, minlength=pt.size)
    return Event(
        n_events=1, n_surfaces=S, offsets=offsets.astype(np.int32),
        loc=loc.astype(np.float32), var=var.astype(np.float32), meas_particle=part.astype(np.int64),
        seed_event=np.zeros(sp.size, np.int32), seed_surface=tr.surface[first].astype(np.int32),
        seed_params=params, seed_cov=_pack_diag(sig5), seed_particle=sp.astype(np.int64),
        seed_truth=truth5, particle_pt=pt, particle_eta=eta, particle_phi=phi, particle_q=q,
        particle_vtx=vtx, particle_nhits=nh, particle_event=np.zeros(pt.size, np.int64), truth=tr)


def concat_events(evs) -> Event:
    """Concatenate single events into one batch (event index = list order)."""
    S = evs[0].n_surfaces
    offs, mo, po = [np.zeros(1, np.int64)], 0, 0
    parts = {k: [] for k in ("loc", "var", "meas_particle", "seed_event", "seed_surface", "seed_params",
                             "seed_cov", "seed_particle", "seed_truth", "particle_pt", "particle_eta",
                             "particle_phi", "particle_q", "particle_vtx", "particle_nhits", "particle_event")}
    tparts = {k: [] for k in ("particle", "surface", "loc", "pos", "dir", "qop", "order")}
    for e, ev in enumerate(evs):
        offs.append(ev.offsets[1:].astype(np.int64) + mo)
        parts["loc"].append(ev.loc)
        parts["var"].append(ev.var)
        parts["meas_particle"].append(np.where(ev.meas_particle >= 0, ev.meas_particle + po, -1))
        parts["seed_event"].append(np.full(ev.n_seeds, e, np.int32))
        parts["seed_surface"].append(ev.seed_surface)
        parts["seed_params"].append(ev.seed_params)
        parts["seed_cov"].append(ev.seed_cov)
        parts["seed_particle"].append(ev.seed_particle + po)
        parts["seed_truth"].append(ev.seed_truth)
        for k in ("particle_pt", "particle_eta", "particle_phi", "particle_q", "particle_vtx", "particle_nhits"):
            parts[k].append(getattr(ev, k))
        parts["particle_event"].append(np.full(ev.particle_pt.size, e, np.int64))
        for k in tparts:
            v = getattr(ev.truth, k)
            tparts[k].append(v + po if k == "particle" else v)
        mo += ev.n_meas
        po += ev.particle_pt.size
    cat = {k: np.concatenate(v) for k, v in parts.items()}
    return Event(n_events=len(evs), n_surfaces=S, offsets=np.concatenate(offs).astype(np.int32),
                 truth=Truth(**{k: np.concatenate(v) for k, v in tparts.items()}), **cat)


def make_batch(det: Detector, rng_seeds, mus, **kw) -> Event:
    return concat_events([make_event(det, s, mu=m, **kw) for s, m in zip(rng_seeds, mus)])
