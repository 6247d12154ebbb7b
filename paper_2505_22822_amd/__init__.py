"""MI355X-native combinatorial Kalman filter (CKF) track finding.

Thin Python binding over libckf.so (include/ckf.h): every step of the track
finder runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch provides device memory and streams.  There is no CPU
fallback: importing works without a GPU, but every call needs libckf.so and
a visible GPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import COUNTER_NAMES

__all__ = ["Geometry", "UniformField", "FieldMap", "Model", "config", "find", "propagate_batch", "kf_update_batch",
           "neighbours", "mlp_forward", "mlp_grad", "mlp_adam", "capture_pairs", "Fitter", "resolve", "CellBatch", "cluster",
           "seed", "CkfError"]


class CkfError(RuntimeError):
    def __init__(self, status, where):
        lib = _abi.load()
        msg = lib.ckf_last_error().decode()
        super().__init__(f"{where}: {_abi.STATUS_NAMES.get(status, status)} ({msg})")
        self.status = status


def _check(rc, where):
    if rc != _abi.CKF_OK:
        raise CkfError(rc, where)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _settle(dev):
    """Wait for the work torch's current stream holds on `dev` (the fills and
    copies that just initialised a call's buffers).  The library's calls run
    on the stream the caller names, which need not be torch's current one
    and is not ordered after it; a buffer is therefore complete before it is
    handed to a call."""
    import torch
    if not torch.cuda.is_current_stream_capturing():
        torch.cuda.current_stream(dev).synchronize()


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def config(**over) -> _abi.Config:
    """Library defaults (ckf_config_default) with overrides."""
    c = _abi.Config()
    _abi.load().ckf_config_default(C.byref(c))
    for k, v in over.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class Geometry:
    """Detector description uploaded once (ckf_geometry_create)."""

    def __init__(self, arrays: dict):
        lib = _abi.load()
        a = {k: np.ascontiguousarray(v) for k, v in arrays.items()}
        self._keep = a
        d = _abi.GeometryDesc(
            a["center"].shape[0], a["center"].ctypes.data, a["rot"].ctypes.data, a["half"].ctypes.data,
            a["thick"].ctypes.data, a["layer"].ctypes.data, a["layer_type"].shape[0], a["layer_type"].ctypes.data,
            a["layer_pos"].ctypes.data, a["layer_lo"].ctypes.data, a["layer_hi"].ctypes.data)
        for k, dt in (("center", np.float32), ("rot", np.float32), ("half", np.float32), ("thick", np.float32),
                      ("layer", np.int32), ("layer_type", np.int32), ("layer_pos", np.float32),
                      ("layer_lo", np.float32), ("layer_hi", np.float32)):
            if a[k].dtype != dt:
                raise TypeError(f"geometry array {k} must be {np.dtype(dt).name}")
        h = C.c_void_p()
        _check(lib.ckf_geometry_create(C.byref(d), C.byref(h)), "ckf_geometry_create")
        self.handle = h
        self.n_surfaces = int(a["center"].shape[0])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _abi.load().ckf_geometry_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


def neighbours(geometry: Geometry):
    """The geometry's neighbour table (ckf_geometry_neighbours): next layers
    [n, 3], anchors [n, 3, 4] = (phi_A, w_A, pitch u, pitch v) and stored
    cell regions [n, 3, 8 * 24] of module ids, -1 padded (numpy)."""
    n = geometry.n_surfaces
    nxt = np.zeros((n, _abi.MAX_NEXT_LAYERS), np.int32)
    anc = np.zeros((n, _abi.MAX_NEXT_LAYERS, 4), np.float32)
    reg = np.zeros((n, _abi.MAX_NEXT_LAYERS, _abi.REGION_U * _abi.REGION_V), np.int32)
    _check(_abi.load().ckf_geometry_neighbours(geometry.handle, nxt.ctypes.data, anc.ctypes.data, reg.ctypes.data),
           "ckf_geometry_neighbours")
    return nxt, anc, reg


class Model:
    """The next-module network packed for the matrix cores (ckf_model_create)
    from FP32 parameters on the device (torch float32 [6752])."""

    def __init__(self, params, stream=None):
        self._check_params(params)
        h = C.c_void_p()
        _check(_abi.load().ckf_model_create(_ptr(params), _stream_handle(stream), C.byref(h)), "ckf_model_create")
        self.handle = h

    @staticmethod
    def _check_params(params):
        import torch
        if params.dtype != torch.float32 or params.numel() != _abi.MLP_PARAMS or not params.is_cuda \
                or not params.is_contiguous():
            raise TypeError("model parameters must be a contiguous float32 device tensor of 6752")

    def update(self, params, stream=None):
        self._check_params(params)
        _check(_abi.load().ckf_model_update(self.handle, _ptr(params), _stream_handle(stream)), "ckf_model_update")

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _abi.load().ckf_model_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


def mlp_forward(model: Model, x, stream=None):
    """Logits [n, 32] (torch, device) of inputs x [n, 7] (float32 device)."""
    import torch
    n = int(x.shape[0])
    out = torch.empty((n, _abi.MLP_OUTPUTS), dtype=torch.float32, device=x.device)
    _check(_abi.load().ckf_mlp_forward(model.handle, _ptr(x.contiguous()), n, _ptr(out), _stream_handle(stream)),
           "ckf_mlp_forward")
    return out


class MlpWorkspace:
    def __init__(self, n, device="cuda"):
        import torch
        nb = C.c_size_t(0)
        _check(_abi.load().ckf_mlp_workspace_size(int(n), C.byref(nb)), "ckf_mlp_workspace_size")
        self.buf = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.n = int(n)


def mlp_grad(params, x, labels, rows=None, n=None, workspace=None, grad=None, loss=None, stream=None):
    """Mean cross-entropy and its gradient (ckf_mlp_grad).  rows: int32
    device tensor (or a raw device address with n) selecting the batch."""
    import torch
    if n is None:
        n = int(rows.shape[0]) if rows is not None and not isinstance(rows, int) else int(x.shape[0])
    ws = workspace if workspace is not None else MlpWorkspace(n, x.device)
    g = grad if grad is not None else torch.empty(_abi.MLP_PARAMS, dtype=torch.float32, device=x.device)
    l = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=x.device)
    rp = C.c_void_p(rows) if isinstance(rows, int) else _ptr(rows)
    _check(_abi.load().ckf_mlp_grad(_ptr(params), _ptr(x), _ptr(labels), rp, int(n), _ptr(ws.buf), ws.buf.numel(),
                                    _ptr(g), _ptr(l), _stream_handle(stream)), "ckf_mlp_grad")
    return g, l


def mlp_adam(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_abi.load().ckf_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), float(lr), float(beta1),
                                    float(beta2), float(eps), _stream_handle(stream)), "ckf_mlp_adam")


def capture_pairs(geometry: Geometry, field, out: dict, cap_pairs: int, stream=None):
    """Training pairs from a Finder's device outputs (made with
    meas_states=True): returns (x [k, 7], label [k], track [k], n_pairs,
    n_dropped) with x/label/track torch device tensors of the captured
    pairs (k = min(n_pairs, cap_pairs))."""
    import torch
    dev = out["offsets"].device
    cap = max(1, int(cap_pairs))
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):  # buffers, the capture and the read-back on one stream
        x = torch.empty((cap, _abi.MLP_INPUTS), dtype=torch.float32, device=dev)
        lab = torch.empty(cap, dtype=torch.int32, device=dev)
        trk = torch.empty(cap, dtype=torch.int32, device=dev)
        counts = torch.zeros(2, dtype=torch.int64, device=dev)
        cap_tracks = int(out["offsets"].numel()) - 1
        lib = _abi.load()
        nb = C.c_size_t(0)
        _check(lib.ckf_capture_workspace_size(cap_tracks, C.byref(nb)), "ckf_capture_workspace_size")
        ws = torch.empty(max(1, int(nb.value)), dtype=torch.uint8, device=dev)
        _check(lib.ckf_capture_pairs(geometry.handle, field.handle, _ptr(out["n_tracks"]), cap_tracks,
                                     _ptr(out["offsets"]), _ptr(out["meas_surface"]), _ptr(out["meas_params"]), cap,
                                     _ptr(x), _ptr(lab), _ptr(trk), _ptr(counts), _ptr(ws), int(nb.value),
                                     _stream_handle(s)), "ckf_capture_pairs")
        c = counts.cpu().numpy()
    k = int(min(c[0], cap))
    return x[:k], lab[:k], trk[:k], int(c[0]), int(c[1])


class FieldMap:
    """A solenoidal (r, z) field map (ckf_field_create_rz) from a dict with
    map [nz, nr, 2] float32 (B_r, B_z), nr, nz, r0, z0, dr, dz."""

    def __init__(self, m: dict):
        v = np.ascontiguousarray(m["map"], np.float32)
        if v.shape != (int(m["nz"]), int(m["nr"]), 2):
            raise ValueError("field map must be [nz, nr, 2]")
        h = C.c_void_p()
        _check(_abi.load().ckf_field_create_rz(v.ctypes.data, int(m["nr"]), int(m["nz"]), float(m["r0"]),
                                               float(m["z0"]), float(m["dr"]), float(m["dz"]), C.byref(h)),
               "ckf_field_create_rz")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _abi.load().ckf_field_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


class UniformField:
    def __init__(self, bx=0.0, by=0.0, bz=2.0):
        h = C.c_void_p()
        _check(_abi.load().ckf_field_create_uniform(bx, by, bz, C.byref(h)), "ckf_field_create_uniform")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _abi.load().ckf_field_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


@dataclass
class Batch:
    """Device-resident inputs of one ckf_find call (torch tensors)."""
    n_events: int
    n_surfaces: int
    offsets: "object"   # int32 [E*S+1]
    loc: "object"       # float32 [n, 2]
    var: "object"       # float32 [n, 2]
    seed_event: "object"    # int32 [k]
    seed_surface: "object"  # int32 [k]
    seed_params: "object"   # float64 [k, 5]
    seed_cov: "object"      # float64 [k, 15]

    @staticmethod
    def from_event(ev, device="cuda"):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        return Batch(ev.n_events, ev.n_surfaces, t(ev.offsets, torch.int32), t(ev.loc, torch.float32),
                     t(ev.var, torch.float32), t(ev.seed_event, torch.int32), t(ev.seed_surface, torch.int32),
                     t(ev.seed_params, torch.float64), t(ev.seed_cov, torch.float64))

    @property
    def n_seeds(self):
        return int(self.seed_params.shape[0])

    @property
    def n_meas(self):
        return int(self.loc.shape[0])


def launch(grid=0, seeds_per_group=0, nodes_per_seed=0, timer=None, waves_per_simd=0) -> _abi.Launch:
    return _abi.Launch(grid, seeds_per_group, nodes_per_seed, timer.handle if timer is not None else None,
                       waves_per_simd)


class KernelTimer:
    """HIP events ckf_find records around its persistent kernel."""

    def __init__(self):
        h = C.c_void_p()
        _check(_abi.load().ckf_timer_create(C.byref(h)), "ckf_timer_create")
        self.handle = h

    def elapsed_ms(self) -> float:
        ms = C.c_float(0)
        _check(_abi.load().ckf_timer_elapsed_ms(self.handle, C.byref(ms)), "ckf_timer_elapsed_ms")
        return float(ms.value)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _abi.load().ckf_timer_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


class Finder:
    """Holds the workspace and output buffers of repeated ckf_find calls on
    one batch shape, so the timed call allocates nothing."""

    def __init__(self, geometry: Geometry, field, batch: Batch, cfg=None, launch_cfg=None, counters=True,
                 model: "Model" = None, meas_states=False, seed_flags=False, tracks_per_seed_cap=None):
        import torch
        self.geometry, self.field, self.batch, self.model = geometry, field, batch, model
        self.cfg = cfg if cfg is not None else config()
        self.launch = launch_cfg if launch_cfg is not None else launch()
        dev = batch.loc.device
        lib = _abi.load()
        nb = C.c_size_t(0)
        _check(lib.ckf_workspace_size(geometry.handle, C.byref(self.cfg), C.byref(self.launch), batch.n_events,
                                      batch.n_seeds, batch.n_meas, C.byref(nb)), "ckf_workspace_size")
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
        # output capacity: one track per seed, or (tracks_per_seed = 0, every
        # finished candidate) tracks_per_seed_cap per seed
        per_seed = 1 if self.cfg.tracks_per_seed == 1 else int(tracks_per_seed_cap or 64)
        n = max(1, batch.n_seeds) * per_seed
        cap_m = n * int(self.cfg.max_steps)
        z = lambda shape, dt: torch.zeros(shape, dtype=dt, device=dev)
        self.out = dict(n_tracks=z(1, torch.int32), offsets=z(n + 1, torch.int32), meas=z(cap_m, torch.int32),
                        params=z((n, 5), torch.float64), cov=z((n, 15), torch.float64), chi2=z(n, torch.float64),
                        ndf=z(n, torch.int32), holes=z(n, torch.int32), seed=z(n, torch.int32),
                        event=z(n, torch.int32), last_surface=z(n, torch.int32), status=z(8, torch.int32),
                        counters=z(len(COUNTER_NAMES), torch.int64) if counters else None,
                        meas_surface=z(cap_m, torch.int32) if meas_states else None,
                        meas_params=z((cap_m, 5), torch.float64) if meas_states else None,
                        seed_flags=z(max(1, batch.n_seeds), torch.int32) if seed_flags else None)
        o = self.out
        self._tracks = _abi.Tracks(n, cap_m, *(_ptr(o[k]) for k in
                                              ("n_tracks", "offsets", "meas", "params", "cov", "chi2", "ndf",
                                               "holes", "seed", "event", "last_surface", "status", "counters",
                                               "meas_surface", "meas_params", "seed_flags")))
        b = batch
        self._meas = _abi.Measurements(b.n_events, b.n_surfaces, b.n_meas, _ptr(b.offsets), _ptr(b.loc),
                                       _ptr(b.var))
        self._seeds = _abi.Seeds(b.n_seeds, _ptr(b.seed_event), _ptr(b.seed_surface), _ptr(b.seed_params),
                                 _ptr(b.seed_cov))
        _settle(dev)

    def enqueue(self, stream=None):
        """One ckf_find on the stream (asynchronous, allocation-free)."""
        lib = _abi.load()
        _check(lib.ckf_find(self.geometry.handle, self.field.handle, C.byref(self._meas), C.byref(self._seeds),
                            C.byref(self.cfg), C.byref(self.launch), self._model_handle(), _ptr(self.workspace),
                            self.workspace.numel(), C.byref(self._tracks), _stream_handle(stream)), "ckf_find")

    def _model_handle(self):
        return self.model.handle if self.model is not None else None

    def capture(self, stream):
        """Capture this call into a hipGraph (ckf_plan_create); later
        launch_graph() replays it.  stream must be a non-default stream."""
        lib = _abi.load()
        h = C.c_void_p()
        _check(lib.ckf_plan_create(self.geometry.handle, self.field.handle, C.byref(self._meas),
                                   C.byref(self._seeds), C.byref(self.cfg), C.byref(self.launch),
                                   self._model_handle(), _ptr(self.workspace), self.workspace.numel(),
                                   C.byref(self._tracks),
                                   _stream_handle(stream), C.byref(h)), "ckf_plan_create")
        self.plan = h

    def launch_graph(self, stream=None):
        _check(_abi.load().ckf_plan_launch(self.plan, _stream_handle(stream)), "ckf_plan_launch")

    def __del__(self):
        h = getattr(self, "plan", None)
        if h is not None and h.value:
            try:
                _abi.load().ckf_plan_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.plan = None

    def status(self):
        return self.out["status"].cpu().numpy()

    def result(self, check=True):
        """Synchronise and return the found tracks as numpy arrays."""
        import torch
        torch.cuda.synchronize()
        st = self.status()
        if check and st[_abi.ST_FLAGS] != 0:
            raise CkfError(3 if st[_abi.ST_FLAGS] & 3 else 2, f"device status flags {st[_abi.ST_FLAGS]}")
        o = {k: v.cpu().numpy() for k, v in self.out.items() if v is not None}
        nt = int(o["n_tracks"][0])
        res = {k: o[k][:nt] for k in ("params", "cov", "chi2", "ndf", "holes", "seed", "event", "last_surface")}
        res["offsets"] = o["offsets"][:nt + 1]
        nm = int(o["offsets"][nt]) if nt > 0 else 0
        res["meas"] = o["meas"][:nm]
        if "meas_surface" in o:
            res["meas_surface"] = o["meas_surface"][:nm]
            res["meas_params"] = o["meas_params"][:nm]
        if "seed_flags" in o:
            res["seed_flags"] = o["seed_flags"][:self.batch.n_seeds]
        res["n_tracks"] = nt
        res["status"] = st
        if "counters" in o:
            res["counters"] = {n: int(o["counters"][i]) for i, n in enumerate(COUNTER_NAMES)}
        return res


SMOOTHERS = {"rts": 0, "two_filter": 1}


class Fitter:
    """Workspace and outputs of repeated ckf_fit calls: the Kalman-filter fit
    of found tracks with the RTS or the two-filter smoother.  `tracks`
    holds device tensors in ckf_find's layout: n_tracks [1], offsets,
    meas, meas_surface, seed (a Finder made with meas_states=True has them
    in .out; see from_finder)."""

    def __init__(self, geometry: Geometry, field, batch: Batch, tracks: dict, cfg=None, smoother="rts"):
        import torch
        if tracks.get("meas_surface") is None:
            raise ValueError("tracks need meas_surface (a Finder made with meas_states=True)")
        self.geometry, self.field, self.batch, self.tracks = geometry, field, batch, tracks
        self.cfg = cfg if cfg is not None else config()
        self.smoother = SMOOTHERS[smoother]
        dev = tracks["offsets"].device
        self.cap_tracks = int(tracks["offsets"].numel()) - 1
        self.cap_meas = int(tracks["meas"].numel())
        nb = C.c_size_t(0)
        _check(_abi.load().ckf_fit_workspace_size(self.cap_meas, C.byref(nb)), "ckf_fit_workspace_size")
        self.workspace = torch.empty(max(1, int(nb.value)), dtype=torch.uint8, device=dev)
        self.params = torch.zeros((self.cap_meas, 5), dtype=torch.float64, device=dev)
        self.cov = torch.zeros((self.cap_meas, 15), dtype=torch.float64, device=dev)
        self.chi2 = torch.zeros(self.cap_tracks, dtype=torch.float64, device=dev)
        self.ok = torch.zeros(self.cap_tracks, dtype=torch.int32, device=dev)
        b = batch
        self._meas = _abi.Measurements(b.n_events, b.n_surfaces, b.n_meas, _ptr(b.offsets), _ptr(b.loc),
                                       _ptr(b.var))
        self._seeds = _abi.Seeds(b.n_seeds, _ptr(b.seed_event), _ptr(b.seed_surface), _ptr(b.seed_params),
                                 _ptr(b.seed_cov))
        _settle(dev)

    @staticmethod
    def from_finder(finder: "Finder", smoother="rts"):
        return Fitter(finder.geometry, finder.field, finder.batch, finder.out, finder.cfg, smoother)

    def enqueue(self, stream=None):
        """One ckf_fit on the stream (asynchronous, allocation-free)."""
        t = self.tracks
        _check(_abi.load().ckf_fit(self.geometry.handle, self.field.handle, C.byref(self._meas),
                                   C.byref(self._seeds), C.byref(self.cfg), _ptr(t["n_tracks"]), self.cap_tracks,
                                   self.cap_meas, _ptr(t["offsets"]), _ptr(t["meas"]), _ptr(t["meas_surface"]),
                                   _ptr(t["seed"]), self.smoother, _ptr(self.workspace), self.workspace.numel(),
                                   _ptr(self.params), _ptr(self.cov), _ptr(self.chi2), _ptr(self.ok),
                                   _stream_handle(stream)), "ckf_fit")

    def result(self):
        """Synchronise and return the smoothed states per measurement
        (aligned with the tracks' meas), chi2 and ok per track (numpy)."""
        import torch
        torch.cuda.synchronize()
        t = self.tracks
        nt = min(int(t["n_tracks"].cpu()[0]), self.cap_tracks)
        off = t["offsets"][:nt + 1].cpu().numpy()
        nm = int(off[-1]) if nt > 0 else 0
        return dict(n_tracks=nt, offsets=off, params=self.params[:nm].cpu().numpy(),
                    cov=self.cov[:nm].cpu().numpy(), chi2=self.chi2[:nt].cpu().numpy(),
                    ok=self.ok[:nt].cpu().numpy())


@dataclass
class CellBatch:
    """Device-resident activated cells in readout order (torch tensors)."""
    n_events: int
    n_surfaces: int
    offsets: "object"   # int32 [E*S+1]
    c0: "object"        # int32 [n]
    c1: "object"        # int32 [n]
    q: "object"         # float32 [n]

    @staticmethod
    def from_cells(c, device="cuda"):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        return CellBatch(c.n_events, c.n_surfaces, t(c.offsets, torch.int32), t(c.c0, torch.int32),
                         t(c.c1, torch.int32), t(c.q, torch.float32))

    @property
    def n_cells(self):
        return int(self.c0.shape[0])


class Clusterer:
    """Workspace and outputs of repeated ckf_cluster calls on one cell-batch
    shape; pitch is a [n_surfaces, 2] float32 device tensor."""

    def __init__(self, geometry: Geometry, cells: CellBatch, pitch, spacepoints=True, cell_cluster=True):
        import torch
        self.geometry, self.cells, self.pitch = geometry, cells, pitch
        dev = cells.c0.device
        self._desc = _abi.CellsDesc(cells.n_events, cells.n_surfaces, cells.n_cells, _ptr(cells.offsets),
                                    _ptr(cells.c0), _ptr(cells.c1), _ptr(cells.q))
        nb = C.c_size_t(0)
        _check(_abi.load().ckf_cluster_workspace_size(C.byref(self._desc), C.byref(nb)), "ckf_cluster_workspace_size")
        self.workspace = torch.empty(max(1, int(nb.value)), dtype=torch.uint8, device=dev)
        n = max(1, cells.n_cells)
        z = lambda shape, dt: torch.zeros(shape, dtype=dt, device=dev)
        self.offsets = z(cells.n_events * cells.n_surfaces + 1, torch.int32)
        self.loc, self.var = z((n, 2), torch.float32), z((n, 2), torch.float32)
        self.spacepoints = z((n, 3), torch.float32) if spacepoints else None
        self.cell_cluster = z(n, torch.int32) if cell_cluster else None
        self.status = z(1, torch.int32)
        _settle(dev)

    def enqueue(self, stream=None):
        _check(_abi.load().ckf_cluster(self.geometry.handle, C.byref(self._desc), _ptr(self.pitch),
                                       _ptr(self.workspace), self.workspace.numel(), _ptr(self.offsets),
                                       _ptr(self.loc), _ptr(self.var), _ptr(self.spacepoints),
                                       _ptr(self.cell_cluster), _ptr(self.status), _stream_handle(stream)),
               "ckf_cluster")

    def measurements(self):
        """The clusters as a Batch-style measurement set (device tensors):
        (offsets, loc, var) views sized to the number of clusters."""
        m = int(self.offsets[-1].item())
        return self.offsets, self.loc[:m], self.var[:m]

    def result(self):
        import torch
        torch.cuda.synchronize()
        m = int(self.offsets[-1].item())
        out = dict(offsets=self.offsets.cpu().numpy(), loc=self.loc[:m].cpu().numpy(), var=self.var[:m].cpu().numpy(),
                   status=int(self.status.item()), n_meas=m)
        if self.spacepoints is not None:
            out["spacepoints"] = self.spacepoints[:m].cpu().numpy()
        if self.cell_cluster is not None:
            out["cell_cluster"] = self.cell_cluster[:self.cells.n_cells].cpu().numpy()
        return out


def cluster(geometry: Geometry, cells: CellBatch, pitch, stream=None):
    """One ckf_cluster call; returns its result (numpy)."""
    c = Clusterer(geometry, cells, pitch)
    c.enqueue(stream)
    return c.result()


def seed(geometry: Geometry, n_events: int, meas_offsets, spacepoints, loc, layers, bz=2.0, cap_seeds=None,
         stream=None, counters=None):
    """Triplet seeding (ckf_seed) on spacepoints in the measurement layout
    (a Clusterer's offsets, spacepoints and loc, device tensors).  layers:
    the seeding layers' geometry ids ordered outwards.  counters: None or a
    device int64 tensor [4] that receives the search's work units
    (CKF_SEED_CNT_*).  Returns a dict of device tensors (event, surface,
    params, cov, spacepoints) sized to the number of seeds, and that
    number."""
    import torch
    lib = _abi.load()
    dev = meas_offsets.device
    n_sp = int(spacepoints.shape[0])
    lay = np.ascontiguousarray(np.asarray(layers, np.int32))
    nl = len(lay)
    nb = C.c_size_t(0)
    _check(lib.ckf_seed_workspace_size(int(n_events), geometry.n_surfaces, n_sp, nl, C.byref(nb)),
           "ckf_seed_workspace_size")
    ws = torch.empty(max(1, int(nb.value)), dtype=torch.uint8, device=dev)
    cap = int(cap_seeds) if cap_seeds is not None else max(1, 2 * n_sp)
    z = lambda shape, dt: torch.zeros(shape, dtype=dt, device=dev)
    out = dict(event=z(cap, torch.int32), surface=z(cap, torch.int32), params=z((cap, 5), torch.float64),
               cov=z((cap, 15), torch.float64), spacepoints=z((cap, 3), torch.int32))
    n = z(1, torch.int32)
    _settle(dev)
    _check(lib.ckf_seed(geometry.handle, int(n_events), _ptr(meas_offsets), n_sp, _ptr(spacepoints), _ptr(loc),
                        lay.ctypes.data_as(C.c_void_p), nl, float(bz), _ptr(ws), ws.numel(), cap, _ptr(n),
                        _ptr(out["event"]), _ptr(out["surface"]), _ptr(out["params"]), _ptr(out["cov"]),
                        _ptr(out["spacepoints"]), _ptr(counters) if counters is not None else None,
                        _stream_handle(stream)), "ckf_seed")
    torch.cuda.synchronize()  # the count is read on the host: wait for the call's stream, whichever it is
    k = int(n.cpu()[0])
    m = min(k, cap)
    return {key: v[:m] for key, v in out.items()}, k


def seed_top_cap(cap=None):
    """ckf_seed_set_top_cap: sets the triplet search's capacity of tops held
    on chip per middle spacepoint (0: always scan each bottom's window; None:
    the maximum, the default).  Returns the maximum."""
    lib = _abi.load()
    mx = C.c_int32(0)
    _check(lib.ckf_seed_set_top_cap(0, C.byref(mx)), "ckf_seed_set_top_cap")  # query the maximum
    _check(lib.ckf_seed_set_top_cap(int(mx.value if cap is None else cap), C.byref(mx)), "ckf_seed_set_top_cap")
    return int(mx.value)


def resolve(tracks: dict, n_meas: int, max_shared=1, stream=None, workspace=None, max_rounds=128, info=None,
            sync=True):
    """Greedy ambiguity resolution (ckf_resolve) of found tracks held as
    device tensors in ckf_find's layout (n_tracks, offsets, meas, chi2, ndf;
    a Finder's .out).  The call itself is asynchronous (its rounds run on the
    device); with sync=True this waits and returns (keep device tensor
    [cap_tracks] int32: 1 kept, 0 removed, -1 invalid; rounds that removed
    tracks), raising if max_rounds did not suffice.  With sync=False it
    returns (keep, info device tensor [2]: rounds, converged)."""
    import torch
    lib = _abi.load()
    dev = tracks["offsets"].device
    cap_tracks = int(tracks["offsets"].numel()) - 1
    cap_meas = int(tracks["meas"].numel())
    if workspace is None:
        nb = C.c_size_t(0)
        _check(lib.ckf_resolve_workspace_size(cap_tracks, int(n_meas), C.byref(nb)), "ckf_resolve_workspace_size")
        workspace = torch.empty(max(1, int(nb.value)), dtype=torch.uint8, device=dev)
    keep = torch.zeros(max(1, cap_tracks), dtype=torch.int32, device=dev)
    if info is None:
        info = torch.zeros(2, dtype=torch.int32, device=dev)
    _settle(dev)
    _check(lib.ckf_resolve(_ptr(tracks["n_tracks"]), cap_tracks, cap_meas, _ptr(tracks["offsets"]),
                           _ptr(tracks["meas"]), int(n_meas), _ptr(tracks["chi2"]), _ptr(tracks["ndf"]),
                           int(max_shared), int(max_rounds), _ptr(workspace), workspace.numel(), _ptr(keep),
                           _ptr(info), _stream_handle(stream)), "ckf_resolve")
    if not sync:
        return keep[:cap_tracks], info
    torch.cuda.synchronize()
    r, conv = (int(x) for x in info.cpu())
    if not conv:
        raise CkfError(3, f"ckf_resolve: {max_rounds} rounds did not remove every bad track")
    return keep[:cap_tracks], r


def find(geometry: Geometry, field, batch: Batch, cfg=None, launch_cfg=None, stream=None, retries=3, model=None,
         meas_states=False, seed_flags=False):
    """Run the track finder on one batch and return the tracks (numpy).
    Retries with a larger history capacity if the device reports it short."""
    lc = launch_cfg if launch_cfg is not None else launch()
    for _ in range(retries + 1):
        f = Finder(geometry, field, batch, cfg, lc, model=model, meas_states=meas_states, seed_flags=seed_flags)
        f.enqueue(stream)
        r = f.result(check=False)
        flags = int(r["status"][_abi.ST_FLAGS])
        if flags & _abi.FLAG_BAD_OFFSETS:
            raise CkfError(2, "measurement offsets are not non-decreasing")
        if flags & _abi.FLAG_NODE_CAPACITY:
            lc = _abi.Launch(lc.grid, lc.seeds_per_group, 2 * (lc.nodes_per_seed or 32), lc.timer,
                             lc.waves_per_simd)
            continue
        if flags:
            raise CkfError(3, f"device status flags {flags}")
        return r
    raise CkfError(3, "history capacity still short after retries")


def propagate_batch(geometry, field, src, params, cov, dst, cfg=None, stream=None):
    """Component call: propagate bound states src -> dst (torch device tensors)."""
    import torch
    cfg = cfg if cfg is not None else config()
    n = int(params.shape[0])
    dev = params.device
    p_out = torch.zeros((n, 5), dtype=torch.float64, device=dev)
    c_out = torch.zeros((n, 15), dtype=torch.float64, device=dev)
    jac = torch.zeros((n, 25), dtype=torch.float64, device=dev)
    path = torch.zeros(n, dtype=torch.float64, device=dev)
    ok = torch.zeros(n, dtype=torch.int32, device=dev)
    _settle(dev)
    _check(_abi.load().ckf_propagate_batch(geometry.handle, field.handle, C.byref(cfg), n, _ptr(src), _ptr(params),
                                           _ptr(cov), _ptr(dst), _ptr(p_out), _ptr(c_out), _ptr(jac), _ptr(path),
                                           _ptr(ok), _stream_handle(stream)), "ckf_propagate_batch")
    return p_out, c_out, jac.view(n, 5, 5), path, ok


def kf_update_batch(params, cov, meas, var, stream=None):
    import torch
    n = int(params.shape[0])
    dev = params.device
    p_out = torch.zeros((n, 5), dtype=torch.float64, device=dev)
    c_out = torch.zeros((n, 15), dtype=torch.float64, device=dev)
    chi2 = torch.zeros(n, dtype=torch.float64, device=dev)
    _settle(dev)
    _check(_abi.load().ckf_kf_update_batch(n, _ptr(params), _ptr(cov), _ptr(meas), _ptr(var), _ptr(p_out),
                                           _ptr(c_out), _ptr(chi2), _stream_handle(stream)), "ckf_kf_update_batch")
    return p_out, c_out, chi2
