"""Python access to the FP64 CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain, slow reference the GPU
library is checked against.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the GPU product
path never does, and the two share no code.

``build()`` compiles ``liboracle.so`` with g++ -O2 -ffp-contract=off.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "oracle.cpp")]

DEFAULT_CONFIG = dict(
    chi2_max=15.0, branches_per_surface=3, max_live_per_seed=10, max_holes=3, min_meas=6,
    max_steps=48, max_rk_steps=100, step_tol=1e-2, step_max=200.0, land_tol=1e-4,
    path_max=4000.0, nav_margin=1.0, mass=0.1056583755, material_on=1, tracks_per_seed=1)


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-Wall", "-o", LIB + ".tmp"] + SRC
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Geometry(C.Structure):
    _fields_ = [("n_surfaces", C.c_int32), ("center", C.c_void_p), ("rot", C.c_void_p),
                ("half", C.c_void_p), ("thick", C.c_void_p), ("layer", C.c_void_p),
                ("n_layers", C.c_int32), ("layer_type", C.c_void_p), ("layer_pos", C.c_void_p),
                ("layer_lo", C.c_void_p), ("layer_hi", C.c_void_p)]


class _Field(C.Structure):
    _fields_ = [("b", C.c_double * 3), ("map", C.c_void_p), ("nr", C.c_int32), ("nz", C.c_int32),
                ("r0", C.c_double), ("z0", C.c_double), ("dr", C.c_double), ("dz", C.c_double)]


def make_field(bfield):
    """A uniform field (3-tuple, tesla) or a map dict (synth.field); returns
    (struct, keep-alive)."""
    if isinstance(bfield, dict):
        m = np.ascontiguousarray(bfield["map"], np.float32)
        f = _Field((C.c_double * 3)(0, 0, 0), m.ctypes.data, int(bfield["nr"]), int(bfield["nz"]),
                   float(bfield["r0"]), float(bfield["z0"]), float(bfield["dr"]), float(bfield["dz"]))
        return f, m
    return _Field((C.c_double * 3)(*bfield), None, 0, 0, 0.0, 0.0, 1.0, 1.0), None


class _Meas(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("n_surfaces", C.c_int32), ("offsets", C.c_void_p),
                ("loc", C.c_void_p), ("var", C.c_void_p)]


class _Seeds(C.Structure):
    _fields_ = [("n_seeds", C.c_int32), ("event", C.c_void_p), ("surface", C.c_void_p),
                ("params", C.c_void_p), ("cov", C.c_void_p)]


class _Config(C.Structure):
    _fields_ = [("chi2_max", C.c_double), ("branches_per_surface", C.c_int32),
                ("max_live_per_seed", C.c_int32), ("max_holes", C.c_int32), ("min_meas", C.c_int32),
                ("max_steps", C.c_int32), ("max_rk_steps", C.c_int32), ("step_tol", C.c_double),
                ("step_max", C.c_double), ("land_tol", C.c_double), ("path_max", C.c_double),
                ("nav_margin", C.c_double), ("mass", C.c_double), ("material_on", C.c_int32),
                ("tracks_per_seed", C.c_int32)]


class _Tracks(C.Structure):
    _fields_ = [("cap_tracks", C.c_int32), ("cap_meas", C.c_int32), ("n_tracks", C.c_int32),
                ("n_meas_total", C.c_int32), ("offsets", C.c_void_p), ("meas", C.c_void_p),
                ("params", C.c_void_p), ("cov", C.c_void_p), ("chi2", C.c_void_p), ("ndf", C.c_void_p),
                ("holes", C.c_void_p), ("seed", C.c_void_p), ("event", C.c_void_p),
                ("last_surface", C.c_void_p), ("meas_surface", C.c_void_p), ("meas_params", C.c_void_p)]


_STAT_NAMES = ("steps", "navigations", "nav_modules", "legs", "legs_failed", "rk_trials", "rk_rejects",
               "chi2_evals", "kf_updates", "ms_updates", "crossed", "holes", "pruned", "finished",
               "mlp_rows", "proposals", "proposal_misses")


class _Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in _STAT_NAMES]


class _Learned(C.Structure):
    _fields_ = [("next", C.c_void_p), ("region", C.c_void_p), ("anchor", C.c_void_p), ("params", C.c_void_p),
                ("min_prob", C.c_double), ("topk", C.c_int32), ("bf16", C.c_int32)]


# causes (bits of the per-seed `near` output) by which an FP32 evaluation of
# the learned proposal can decide otherwise than the oracle's FP64 one
NEAR_CONF, NEAR_BF16, NEAR_EDGE, NEAR_RANK = 1, 2, 4, 8

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.orc_ckf_find.restype = C.c_int
        _lib.orc_propagate.restype = C.c_int
        _lib.orc_propagate_free.restype = C.c_int
        _lib.orc_kf_update.restype = C.c_int
        _lib.orc_trace.restype = C.c_int
        _lib.orc_navigate.restype = C.c_int
        _lib.orc_navigate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                      C.c_uint64, C.c_double, C.c_void_p, C.c_void_p]
        _lib.orc_scatter.restype = C.c_int
        _lib.orc_ckf_find_learned.restype = C.c_int
        _lib.orc_mlp_forward.restype = C.c_int
        _lib.orc_mlp_forward.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p]
        _lib.orc_learned_propose.restype = C.c_int
        _lib.orc_learned_propose.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                             C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p]
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


class Inputs:
    """Keeps contiguous copies alive while the ctypes structs point at them."""

    def __init__(self, geom: dict, bfield=(0.0, 0.0, 2.0), event=None):
        self.keep = []
        g = {k: np.ascontiguousarray(v) for k, v in geom.items()}
        self.keep.append(g)
        self.geom = _Geometry(g["center"].shape[0], _p(g["center"]), _p(g["rot"]), _p(g["half"]),
                              _p(g["thick"]), _p(g["layer"]), g["layer_type"].shape[0],
                              _p(g["layer_type"]), _p(g["layer_pos"]), _p(g["layer_lo"]), _p(g["layer_hi"]))
        self.field, fkeep = make_field(bfield)
        self.keep.append(fkeep)
        if event is not None:
            self.set_event(event)

    def set_event(self, ev, seeds=None):
        off = np.ascontiguousarray(ev.offsets, np.int32)
        loc = np.ascontiguousarray(ev.loc, np.float32)
        var = np.ascontiguousarray(ev.var, np.float32)
        se = np.ascontiguousarray(ev.seed_event, np.int32)
        ss = np.ascontiguousarray(ev.seed_surface, np.int32)
        sp = np.ascontiguousarray(ev.seed_params, np.float64)
        sc = np.ascontiguousarray(ev.seed_cov, np.float64)
        if seeds is not None:
            se, ss, sp, sc = (np.ascontiguousarray(a[seeds]) for a in (se, ss, sp, sc))
        self.keep.append((off, loc, var, se, ss, sp, sc))
        self.meas = _Meas(ev.n_events, ev.n_surfaces, _p(off), _p(loc), _p(var))
        self.seeds = _Seeds(sp.shape[0], _p(se), _p(ss), _p(sp), _p(sc))
        self.n_seeds = sp.shape[0]


def make_config(**over):
    d = dict(DEFAULT_CONFIG)
    d.update(over)
    return _Config(**d), d


class LearnedInputs:
    """The learned proposal's inputs for the oracle: the neighbour table of
    the whole detector (``oracle.learned.neighbour_table``), the network
    parameters and the use rule; keeps the arrays alive."""

    def __init__(self, table, params, min_prob=0.95, topk=3, bf16=True):
        nxt, reg, anc = table
        self.next = np.ascontiguousarray(nxt, np.int32)
        self.region = np.ascontiguousarray(reg, np.int32)
        self.anchor = np.ascontiguousarray(anc, np.float64)
        self.params = np.ascontiguousarray(params, np.float32)
        assert self.params.shape == (6752,)
        self.struct = _Learned(_p(self.next), _p(self.region), _p(self.anchor), _p(self.params),
                               float(min_prob), int(topk), int(bool(bf16)))


def ckf_find(inp: Inputs, n_threads=0, cap_tracks=None, cap_meas=None, learned: LearnedInputs = None, **cfg):
    """Run the oracle; returns a dict of numpy arrays (tracks in seed order).
    With `learned`, the search uses the learned proposal and the result also
    holds per seed ``near`` (the NEAR_* causes met) and ``differs`` (a used
    proposal listed differently from the geometric lookup)."""
    conf, _ = make_config(**cfg)
    n = inp.n_seeds
    mult = 1 if conf.tracks_per_seed == 1 else 64
    cap_t = cap_tracks or max(1, n * mult)
    cap_m = cap_meas or max(1, cap_t * 64)
    out = dict(offsets=np.zeros(cap_t + 1, np.int32), meas=np.zeros(cap_m, np.int32),
               params=np.zeros((cap_t, 5)), cov=np.zeros((cap_t, 15)), chi2=np.zeros(cap_t),
               ndf=np.zeros(cap_t, np.int32), holes=np.zeros(cap_t, np.int32),
               seed=np.zeros(cap_t, np.int32), event=np.zeros(cap_t, np.int32),
               last_surface=np.zeros(cap_t, np.int32), meas_surface=np.zeros(cap_m, np.int32),
               meas_params=np.zeros((cap_m, 5)))
    tr = _Tracks(cap_t, cap_m, 0, 0, *(_p(out[k]) for k in
                                        ("offsets", "meas", "params", "cov", "chi2", "ndf", "holes",
                                         "seed", "event", "last_surface", "meas_surface", "meas_params")))
    st = _Stats()
    if learned is None:
        rc = lib().orc_ckf_find(C.byref(inp.geom), C.byref(inp.field), C.byref(inp.meas), C.byref(inp.seeds),
                                C.byref(conf), int(n_threads), C.byref(tr), C.byref(st))
    else:
        near = np.zeros(max(1, n), np.int32)
        differs = np.zeros(max(1, n), np.int32)
        rc = lib().orc_ckf_find_learned(C.byref(inp.geom), C.byref(inp.field), C.byref(inp.meas),
                                        C.byref(inp.seeds), C.byref(conf), C.byref(learned.struct),
                                        int(n_threads), C.byref(tr), C.byref(st), _p(near), _p(differs))
    if rc != 0:
        raise RuntimeError(f"orc_ckf_find failed with status {rc} (tracks {tr.n_tracks}, meas {tr.n_meas_total})")
    nt, nm = tr.n_tracks, tr.n_meas_total
    per_meas = ("meas", "meas_surface", "meas_params")
    res = {k: v[:nt] for k, v in out.items() if k != "offsets" and k not in per_meas}
    res["offsets"] = out["offsets"][:nt + 1]
    for k in per_meas:
        res[k] = out[k][:nm]
    res["n_tracks"] = nt
    res["stats"] = {k: int(getattr(st, k)) for k in _STAT_NAMES}
    if learned is not None:
        res["near"] = near[:n]
        res["differs"] = differs[:n]
    return res


def mlp_forward(params, x, bf16=True):
    """Network logits [n, 32] of inputs x [n, 7] (the oracle's C++ pass)."""
    pr = np.ascontiguousarray(params, np.float32)
    xx = np.ascontiguousarray(x, np.float64).reshape(-1, 7)
    out = np.zeros((xx.shape[0], 32))
    rc = lib().orc_mlp_forward(_p(pr), int(bool(bf16)), xx.shape[0], _p(xx), _p(out))
    if rc != 0:
        raise RuntimeError("orc_mlp_forward failed")
    return out


def learned_propose(inp: Inputs, learned: LearnedInputs, surface, layer, X, T, qop):
    """One proposal: None when the network does not run, else a dict with the
    window cell, the unrounded input, the summed top-k probability, the three
    most probable outputs, the proposed modules, `used` and the NEAR_* causes."""
    Xa = np.ascontiguousarray(X, np.float64)
    Ta = np.ascontiguousarray(T, np.float64)
    cell = np.zeros(2, np.int32)
    feat = np.zeros(7)
    conf = C.c_double(0)
    cls = np.zeros(3, np.int32)
    mods = np.zeros(3, np.int32)
    near = C.c_int32(0)
    rc = lib().orc_learned_propose(C.byref(inp.geom), C.byref(learned.struct), int(surface), int(layer), _p(Xa),
                                   _p(Ta), float(qop), _p(cell), _p(feat), C.byref(conf), _p(cls), _p(mods),
                                   C.byref(near))
    if rc < 0:
        return None
    return dict(cell=cell, features=feat, conf=conf.value, classes=cls, modules=mods, used=bool(rc),
                near=near.value)


def propagate(inp: Inputs, src, params, cov, dst, **cfg):
    conf, _ = make_config(**cfg)
    p = np.ascontiguousarray(params, np.float64)
    c = np.ascontiguousarray(cov, np.float64)
    po, co, jac, path = np.zeros(5), np.zeros(15), np.zeros(25), C.c_double(0)
    rc = lib().orc_propagate(C.byref(inp.geom), C.byref(inp.field), C.byref(conf), int(src), _p(p), _p(c),
                             int(dst), _p(po), _p(co), _p(jac), C.byref(path))
    if rc != 0:
        return None
    return po, co, jac.reshape(5, 5), path.value


def propagate_free(bfield, free, center, normal, **cfg):
    conf, _ = make_config(**cfg)
    f, _keep = make_field(bfield)
    fi = np.ascontiguousarray(free, np.float64)
    cc = np.ascontiguousarray(center, np.float64)
    nn = np.ascontiguousarray(normal, np.float64)
    fo, path = np.zeros(7), C.c_double(0)
    rc = lib().orc_propagate_free(C.byref(f), C.byref(conf), _p(fi), _p(cc), _p(nn), _p(fo), C.byref(path))
    if rc != 0:
        return None
    return fo, path.value


def kf_update(params, cov, meas, var):
    p = np.ascontiguousarray(params, np.float64)
    c = np.ascontiguousarray(cov, np.float64)
    m = np.ascontiguousarray(meas, np.float64)
    v = np.ascontiguousarray(var, np.float64)
    po, co, x2 = np.zeros(5), np.zeros(15), C.c_double(0)
    rc = lib().orc_kf_update(_p(p), _p(c), _p(m), _p(v), _p(po), _p(co), C.byref(x2))
    assert rc == 0
    return po, co, x2.value


def trace(inp: Inputs, surface, params, cap=64, **cfg):
    conf, _ = make_config(**cfg)
    p = np.ascontiguousarray(params, np.float64)
    vis, cr, po = np.zeros(cap, np.int32), np.zeros(cap, np.int32), np.zeros((cap, 5))
    n = lib().orc_trace(C.byref(inp.geom), C.byref(inp.field), C.byref(conf), int(surface), _p(p), int(cap),
                        _p(vis), _p(cr), _p(po))
    return vis[:n], cr[:n], po[:n]


def navigate(inp: Inputs, surface, params, mask, path=0.0, **cfg):
    """(next layer or -1, listed modules) from bound parameters on surface."""
    conf, _ = make_config(**cfg)
    p = np.ascontiguousarray(params, np.float64)
    lst, n = np.zeros(8, np.int32), C.c_int32(0)
    L = lib().orc_navigate(C.addressof(inp.geom), C.addressof(inp.field), C.addressof(conf), int(surface),
                           p.ctypes.data, C.c_uint64(int(mask)), float(path), lst.ctypes.data, C.addressof(n))
    return L, lst[:n.value].tolist()


def seed_list(inp: Inputs, surface, params, **cfg):
    conf, _ = make_config(**cfg)
    p = np.ascontiguousarray(params, np.float64)
    lst = np.zeros(8, np.int32)
    n = lib().orc_seed_list(C.byref(inp.geom), C.byref(inp.field), C.byref(conf), int(surface), _p(p), _p(lst))
    return lst[:n].tolist()


def scatter(inp: Inputs, surface, params, cov, **cfg):
    conf, _ = make_config(**cfg)
    p = np.ascontiguousarray(params, np.float64)
    c = np.array(cov, np.float64)
    assert lib().orc_scatter(C.byref(inp.geom), C.byref(conf), int(surface), _p(p), _p(c)) == 0
    return c


PACKED = [(i, j) for i in range(5) for j in range(i, 5)]


def unpack_cov(c15):
    c15 = np.asarray(c15)
    M = np.zeros(c15.shape[:-1] + (5, 5))
    for k, (i, j) in enumerate(PACKED):
        M[..., i, j] = c15[..., k]
        M[..., j, i] = c15[..., k]
    return M


def pack_cov(M):
    M = np.asarray(M)
    return np.stack([M[..., i, j] for (i, j) in PACKED], -1)


def field_eval(bfield, points, grad=False):
    """The oracle's field (and gradient of the interpolant) at points [n, 3]."""
    f, keep = make_field(bfield)
    p = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
    B = np.zeros_like(p)
    G = np.zeros((p.shape[0], 3, 3)) if grad else None
    rc = lib().orc_field_eval(C.byref(f), p.shape[0], _p(p), _p(B), _p(G))
    del keep
    if rc != 0:
        raise RuntimeError("orc_field_eval failed")
    return (B, G) if grad else B
