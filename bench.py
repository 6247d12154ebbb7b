"""Throughput of CKF track finding on one MI355X: learned proposal vs plain.

Workload: a batch of 64 synthetic mu = 200 events (about 10k seeds and 80k
measurements each) in the barrel + endcap detector with 1 % X0 per module
and a uniform 2 T field, found in one persistent launch.  A step is one
ckf_find over the whole batch with inputs already resident in HBM, replayed
from a hipGraph.

Both forms of the search run on the same batch: the plain geometric
navigation, and the learned form, whose next-module network is trained on
the GPU at start-up (pairs captured from the plain search on separate
training events, seeds 5000 + i; Adam, 20 epochs, batch 4096).  `value` is
the learned form's tracks/s; the plain form's figures and both finding
efficiencies (double matching, paper section 3.1) are in the same line.

Prints one JSON line: tracks/s, the roofline object of the dominant kernel
(k_ckf of the form `value` measures: algorithmic FP32 + FP64 (+ bf16 MFMA)
work from the kernel's own work-unit counters over its average duration
measured with HIP events on its stream), and the oracle timed on the host's
cores on a bounded sample of the same events.
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit counted by the kernel (FP32 flop, FP64 flop),
# counted from the arithmetic each unit performs.
UNIT_FLOPS = {
    "rk_trials": (505, 0),      # RKN4 stage algebra + 3 tangent columns + landing prediction
    "legs": (300, 400),         # bound->free, free->bound Jacobian (FP32); J C J^T (FP64)
    "navigations": (300, 0),    # helix set-up and envelope crossings
    "nav_modules": (60, 0),     # listing test of one candidate module
    "chi2_evals": (0, 15),      # 2x2 innovation chi2
    "kf_updates": (0, 450),     # gain + Joseph update
    "ms_updates": (40, 4),      # Highland width (FP32), covariance increment (FP64)
    "mlp_rows": (90, 0),        # network input (30) and softmax/top-3 of one row (60)
}
MFMA_FLOP_PER_BLOCK = 28 * 16 * 16 * 16 * 2  # one 16-row network pass: 28 bf16 16x16x16 MFMAs
# HBM bytes per launch of the track-finding kernel from the FETCH_SIZE and
# WRITE_SIZE counters (scaled by a plain copy's factors 2.0 and 1.0), keyed
# by (form, grid, seeds per group, waves per SIMD): the pools make the
# traffic depend on the launch shape.  Each value carries the hash of the
# library sources it was measured on (code_hash()); roofline_of reports it
# only while the sources hash the same, so a changed kernel prints null
# until it is profiled again.  Source: profiles/k_ckf_mu200x64_hbm_traffic.md.
MEASURED_TRAFFIC = {
    ("plain", 2048, 48, 2): (22.94e9, "2da49482bb6e3ae2"),
    ("learned", 2048, 48, 2): (23.85e9, "2da49482bb6e3ae2"),
    ("learned", 4096, 48, 2): (23.55e9, "2da49482bb6e3ae2"),
}
# SIMT efficiency of the same launches, SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU): the share of
# lanes a VALU instruction finds active, same keys and hashes.  Source: profiles/k_ckf_mu200x64_sq_counters.md.
MEASURED_SIMT = {
    ("plain", 2048, 48, 2): (0.385, "2da49482bb6e3ae2"),
    ("learned", 2048, 48, 2): (0.339, "2da49482bb6e3ae2"),
    ("learned", 4096, 48, 2): (0.339, "2da49482bb6e3ae2"),
}
# HBM bytes per ckf_fit call (k_fit and its sort kernels) on the 64 x mu=200
# batch's plain-search tracks (per smoother), and per call of ckf_cluster, ckf_seed and ckf_resolve on
# the same batch, summed over the call's kernels, same counters and
# factors, keyed by the sizes of the call and carrying the source hash like
# the values above.  Sources: profiles/k_fit_mu200x64.md,
# profiles/k_cl_k_sd_k_res_mu200x64_hbm_traffic.md.
FIT_TRAFFIC = {      # (tracks, measurements, smoother) -> (bytes, hash)
    (560805, 4620862, "rts"): (6.894e9, "2da49482bb6e3ae2"),
    (560805, 4620862, "two_filter"): (8.625e9, "2da49482bb6e3ae2"),
}
CLUSTER_TRAFFIC = {  # (cells, clusters) -> (bytes, hash)
    (9783486, 5260424): (1.252e9, "2da49482bb6e3ae2"),
}
SEED_TRAFFIC = {     # (spacepoints, seeds) -> (bytes, hash)
    (5260424, 2312126): (3.954e9, "2da49482bb6e3ae2"),
}
RESOLVE_TRAFFIC = {  # (tracks, measurements) -> (bytes, hash)
    (560805, 4620862): (1.495e9, "2da49482bb6e3ae2"),
}
# Learned proposal: the configured threshold, the candidates the bench
# chooses from on held-out events, and the equal-efficiency allowance
# (absolute finding efficiency) with the margin the choice keeps below it.
CFG_MIN_PROB = 0.95
THRESHOLDS = (0.95, 0.97, 0.98, 0.99, 0.995)
EFF_ALLOWANCE = 0.005
EFF_MARGIN = 0.001
PEAK_FP32 = 157.3e12  # MI355X vector FP32, FLOP/s
PEAK_FP64 = 78.6e12   # MI355X vector FP64, FLOP/s
PEAK_BF16 = 2.5e15    # MI355X dense bf16 MFMA, FLOP/s


def code_hash():
    """First 16 hex digits of the SHA-256 over the library's HIP and C++
    sources (file names and contents, in name order)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2505_22822_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured(table, key):
    """A measured counter value of `table` for `key`, or None when none was
    measured for it or the sources changed since."""
    v = table.get(key)
    if v is None or v[1] != code_hash():
        return None
    return v[0]


def _gen(args):
    from synth import barrel_endcap, make_event
    seed, mu, cells = args[:3]
    field_map = len(args) > 3 and args[3]
    det = barrel_endcap()
    if field_map:
        from synth.field import solenoid_field
        ev = make_event(det, seed, mu=mu, field=solenoid_field)
    else:
        ev = make_event(det, seed, mu=mu)
    if not cells:
        return ev
    from synth.cells import make_cells
    return ev, make_cells(det, ev, seed + 100000)


def make_events(seeds, mu, workers, cells=False, field_map=False):
    """Events (and, with cells=True, their detector cells) generated in
    parallel; mu is one pileup for all events or one per event; field_map:
    truth integrated through the solenoid field instead of helices in 2 T.
    Returns (events, concatenated batch[, concatenated cells])."""
    from synth import concat_events
    mus = np.broadcast_to(np.asarray(mu, dtype=float), (len(seeds),))
    jobs = [(s, float(m), cells, field_map) for s, m in zip(seeds, mus)]
    if workers > 1:
        import multiprocessing as mp
        # closed and joined, not terminated: the workers end on their own
        pool = mp.get_context("fork").Pool(workers)
        try:
            out = pool.map(_gen, jobs)
        finally:
            pool.close()
            pool.join()
    else:
        out = [_gen(j) for j in jobs]
    if not cells:
        return out, concat_events(out)
    from synth.cells import concat_cells
    evs = [e for e, _ in out]
    return evs, concat_events(evs), concat_cells([c for _, c in out])


# The uneven batch: 64 events whose pileup is drawn uniformly in [20, 200]
# (about 1k to 10k seeds each), found in one persistent launch.
UNEVEN_SEEDS = [6100 + i for i in range(64)]


def uneven_mus(n, seed=6100):
    """Pileup of each event of the uneven batch: U[20, 200] from PCG64(seed)."""
    return np.random.Generator(np.random.PCG64(seed)).uniform(20.0, 200.0, n)


def efficiency(ev, r):
    """Paper section 3.1: a track is double-matched to the particle that
    contributes N of its Nt measurements (of Np it has) if N > Nt/2 and
    N > Np/2 and the seed came from that particle.  Efficiency: fraction of
    reconstructible seeded particles (pT > 0.5 GeV, vertex |z| < 500 mm and
    r < 200 mm) with a double-matched track."""
    nt = int(r["n_tracks"])
    off = r["offsets"]
    meas = r["meas"]
    if nt == 0:
        return 0.0
    tid = np.repeat(np.arange(nt), np.diff(off))
    part = ev.meas_particle[meas]
    ok = part >= 0
    P = int(ev.particle_pt.shape[0]) + 1
    uk, cnt = np.unique(tid[ok].astype(np.int64) * P + part[ok], return_counts=True)
    t_of, p_of = uk // P, uk % P
    order = np.lexsort((-cnt, t_of))
    first = order[np.r_[True, t_of[order][1:] != t_of[order][:-1]]]
    tr, maj, N = t_of[first], p_of[first], cnt[first]
    Nt = np.diff(off)[tr]
    Np = ev.particle_nhits[maj]
    sp = ev.seed_particle[r["seed"][tr]]
    matched = (N > Nt / 2) & (N > Np / 2) & (maj == sp)
    vtx = ev.particle_vtx
    recon = (ev.particle_pt > 0.5) & (np.abs(vtx[:, 2]) < 500) & (np.hypot(vtx[:, 0], vtx[:, 1]) < 200)
    seeded = np.zeros(P - 1, bool)
    seeded[ev.seed_particle] = True
    den = recon & seeded
    found = np.zeros(P - 1, bool)
    found[maj[matched]] = True
    return float((found & den).sum() / max(1, den.sum()))


def cpu_single_thread(batch, n_seeds):
    """The oracle on one thread: the first n_seeds seeds of the batch."""
    import oracle
    from synth import barrel_endcap
    det = barrel_endcap()
    inp = oracle.Inputs(det.as_arrays(), (0, 0, 2.0))
    sel = np.arange(min(n_seeds, batch.n_seeds))
    inp.set_event(batch, seeds=sel)
    t0 = time.perf_counter()
    r = oracle.ckf_find(inp, n_threads=1)
    dt = time.perf_counter() - t0
    return dict(value=r["n_tracks"] / dt, unit="tracks/s", cores=1,
                sample=f"first {len(sel)} seeds of the batch ({r['n_tracks']} tracks) in {dt:.2f} s")


def cpu_baseline(batch, n_events):
    import oracle
    from synth import barrel_endcap
    oracle.build(force=not os.path.exists(oracle.LIB))
    det = barrel_endcap()
    inp = oracle.Inputs(det.as_arrays(), (0, 0, 2.0))
    sel = np.nonzero(batch.seed_event < n_events)[0]
    inp.set_event(batch, seeds=sel)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    r = oracle.ckf_find(inp, n_threads=cores)
    dt = time.perf_counter() - t0
    return dict(value=r["n_tracks"] / dt, unit="tracks/s", cores=cores, kind="oracle",
                sample=f"first {n_events} of the {batch.n_events} events ({len(sel)} seeds, "
                       f"{r['n_tracks']} tracks) in {dt:.2f} s")


def measure(ckf, geo, fld, b, shape, steps, warmup, stream, model=None, audit=False, cfg=None):
    """Counting run (work units), eager runs timed by the library's kernel
    timer, then the hipGraph-captured call replayed `steps` times."""
    import torch
    lc = lambda timer=None: ckf.launch(shape["grid"], shape["seeds_per_group"], 0, timer, shape["waves_per_simd"])
    cfg = cfg if cfg is not None else ckf.config()
    counting = ckf.Finder(geo, fld, b, cfg, lc(), counters=True, model=model, seed_flags=audit)
    counting.enqueue(stream)
    rc = counting.result()
    del counting
    timer = ckf.KernelTimer()
    eager = ckf.Finder(geo, fld, b, cfg, lc(timer), counters=False, model=model)
    kernel_ms = []
    for i in range(warmup + steps):
        eager.enqueue(stream)
        ms = timer.elapsed_ms()
        if i >= warmup:
            kernel_ms.append(ms)
    r = eager.result()
    assert r["n_tracks"] == rc["n_tracks"] and np.array_equal(r["meas"], rc["meas"]), "variants disagree"
    del eager
    finder = ckf.Finder(geo, fld, b, cfg, lc(), counters=False, model=model)
    finder.capture(stream)
    for _ in range(warmup):
        finder.launch_graph(stream)
    stream.synchronize()
    t_start, t_stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(steps):
        finder.launch_graph(stream)
    t_stop.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_stop)
    rg = finder.result()
    assert rg["n_tracks"] == r["n_tracks"] and np.array_equal(rg["meas"], r["meas"]), "graph replay disagrees"
    ms_per_step = total_ms / steps
    return dict(result=r, counters=rc["counters"], seed_flags=rc.get("seed_flags"), kernel_ms=float(np.mean(kernel_ms)),
                ms_per_step=ms_per_step, tracks_per_s=r["n_tracks"] / (ms_per_step * 1e-3))


def _find_once(ckf, geo, fld, b, shape, model=None, cfg=None):
    """One uninstrumented ckf_find; the result arrays."""
    f = ckf.Finder(geo, fld, b, cfg or ckf.config(),
                   ckf.launch(shape["grid"], shape["seeds_per_group"], 0, None, shape["waves_per_simd"]),
                   counters=False, model=model)
    f.enqueue()
    return f.result()


def measure_end_to_end(ckf, geo, fld, batch, shape, stream, reps):
    """The whole batch from host memory: the inputs (measurement offsets,
    loc, var; seed events, surfaces, parameters, covariances) copied from
    pinned host buffers to the device, the captured ckf_find, the outputs
    (track CSR and per-track arrays) copied back to pinned host buffers;
    wall time of the sequence on one stream, mean over reps."""
    import torch
    host = ckf.Batch.from_event(batch, device="cpu")
    names = ("offsets", "loc", "var", "seed_event", "seed_surface", "seed_params", "seed_cov")
    pinned = {k: getattr(host, k).pin_memory() for k in names}
    dev = ckf.Batch.from_event(batch)
    finder = ckf.Finder(geo, fld, dev, ckf.config(),
                        ckf.launch(shape["grid"], shape["seeds_per_group"], 0, None, shape["waves_per_simd"]),
                        counters=False)
    finder.capture(stream)
    outs = ("n_tracks", "offsets", "meas", "params", "cov", "chi2", "ndf", "holes", "seed", "event", "last_surface",
            "status")
    back = {k: torch.empty_like(finder.out[k], device="cpu").pin_memory() for k in outs}
    bytes_in = sum(t.numel() * t.element_size() for t in pinned.values())
    bytes_out = sum(t.numel() * t.element_size() for t in back.values())
    times = []
    for i in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for k in names:
                getattr(dev, k).copy_(pinned[k], non_blocking=True)
            finder.launch_graph(stream)
            for k in outs:
                back[k].copy_(finder.out[k], non_blocking=True)
        stream.synchronize()
        if i > 0:
            times.append((time.perf_counter() - t0) * 1e3)
    nt = int(back["n_tracks"][0])
    ms = float(np.mean(times))
    return dict(ms=round(ms, 4), tracks=nt, tracks_per_s=round(nt / (ms * 1e-3), 1), bytes_in=int(bytes_in),
                bytes_out=int(bytes_out), reps=reps,
                note="wall time: pinned host inputs -> device, the captured ckf_find, outputs -> pinned host "
                     "(output arrays at their full capacity)")


# Kalman-filter fit, per measurement (FP32 flop, FP64 flop): the forward
# filter's leg (bound->free, free->bound Jacobian; J C J^T), chi2, update and
# scattering; the RTS step (F C_k|k, Cholesky of C_k+1|k and its solve for
# A^T, the state and the A (C' - C) A^T products); the two-filter step (the
# backward leg, its update and scattering, the Cholesky solve of the
# combination and its products).  The legs' RKN4 trials are priced at the
# search's measured trials per leg.
# FP64 flop per work unit of ckf_seed's triplet search (CKF_SEED_CNT_*),
# counted from the arithmetic of its cuts: an (M, T) doublet (radius
# difference, cot, the two azimuth products and their bound) 10, a (B, M)
# doublet 12 (its line's z at r = 0 too), a (B, T) cot comparison 1, a
# triplet 44 (the circle through the three points, its radius and the
# distance of closest approach).
SEED_FLOPS = (10, 12, 1, 44)
FIT_FORWARD = (300 + 40, 400 + 15 + 450 + 4)
FIT_RTS = (0, 1100)
FIT_TWO = (300 + 40, 400 + 450 + 4 + 780)


def measure_fit(ckf, geo, fld, b, shape, stream, reps, trials_per_leg):
    """Both smoothers on the plain search's tracks of the batch: device time
    of one ckf_fit launch (HIP events on the launch stream, mean of reps),
    fitted fraction and the algorithmic rate."""
    import torch
    finder = ckf.Finder(geo, fld, b, ckf.config(), ckf.launch(**shape), counters=False, meas_states=True)
    with torch.cuda.stream(stream):
        finder.enqueue(stream)
    r = finder.result()
    n_t, n_m = r["n_tracks"], len(r["meas"])
    out = dict(tracks=n_t, measurements=n_m)
    for name in ("rts", "two_filter"):
        f = ckf.Fitter.from_finder(finder, name)
        f.enqueue(stream)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            f.enqueue(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        g = f.result()
        rk = 505 * trials_per_leg
        if name == "rts":
            f32 = n_m * (FIT_FORWARD[0] + rk)
            f64 = n_m * (FIT_FORWARD[1] + FIT_RTS[1])
        else:
            f32 = n_m * (FIT_FORWARD[0] + FIT_TWO[0] + 2 * rk)
            f64 = n_m * (FIT_FORWARD[1] + FIT_TWO[1])
        frac = (f32 / PEAK_FP32 + f64 / PEAK_FP64) / (ms * 1e-3)
        traffic = _measured(FIT_TRAFFIC, (n_t, n_m, name))
        out[name] = dict(tracks_per_s=round(n_t / (ms * 1e-3), 1), kernel_ms=round(ms, 4),
                         fitted=round(float(np.mean(g["ok"] == 1)), 6),
                         roofline=dict(bound="alu", achieved=round(frac * PEAK_FP32 / 1e12, 3),
                                       peak=PEAK_FP32 / 1e12, unit="TFLOP/s", frac=round(frac, 5), traffic=traffic,
                                       kernel="k_fit", fp32_flop=int(f32), fp64_flop=int(f64),
                                       hbm_tb_per_s=round(traffic / (ms * 1e-3) / 1e12, 3) if traffic else None))
    out["_finder"] = finder
    return out


def _majority(ev, r):
    """Per track with a particle hit: (track, majority particle, N, Nt, Np)."""
    nt, off, meas = int(r["n_tracks"]), r["offsets"], r["meas"]
    tid = np.repeat(np.arange(nt), np.diff(off))
    part = ev.meas_particle[meas]
    ok = part >= 0
    P = int(ev.particle_pt.shape[0]) + 1
    uk, cnt = np.unique(tid[ok].astype(np.int64) * P + part[ok], return_counts=True)
    t_of, p_of = uk // P, uk % P
    order = np.lexsort((-cnt, t_of))
    first = order[np.r_[True, t_of[order][1:] != t_of[order][:-1]]] if len(order) else order
    tr, maj, N = t_of[first], p_of[first], cnt[first]
    return tr, maj, N, np.diff(off)[tr], ev.particle_nhits[maj]


def track_rates(ev, r, keep=None):
    """Paper section 4: fake tracks (no particle double-matched) and
    duplicate tracks (double-matched to a particle that another kept track
    already matches), as fractions of the kept tracks."""
    nt = int(r["n_tracks"])
    kept = np.ones(nt, bool) if keep is None else (keep[:nt] == 1)
    tr, maj, N, Nt, Np = _majority(ev, r)
    good = (N > Nt / 2) & (N > Np / 2) & kept[tr]
    n = int(kept.sum())
    matched = int(good.sum())
    distinct = int(np.unique(maj[good]).size)
    return dict(tracks=n, fake_rate=round((n - matched) / max(1, n), 6),
                duplicate_rate=round((matched - distinct) / max(1, n), 6))


def kept_tracks(r, keep):
    """The result dict restricted to the kept tracks (for the efficiency)."""
    nt = int(r["n_tracks"])
    k = np.nonzero(keep[:nt] == 1)[0]
    n = np.diff(r["offsets"])[k]
    off = np.zeros(len(k) + 1, np.int64)
    off[1:] = np.cumsum(n)
    idx = np.concatenate([np.arange(r["offsets"][t], r["offsets"][t + 1]) for t in k]) if len(k) else np.zeros(0, int)
    return dict(n_tracks=len(k), offsets=off, meas=r["meas"][idx], seed=r["seed"][k])


def measure_resolve(ckf, finder, ev, stream, reps=3, max_rounds=8):
    """Ambiguity resolution of a finder's tracks: wall time of the call (its
    rounds run on the device, bounded by max_rounds, with no host
    synchronisation), rounds, removed tracks, fake and duplicate rates and
    efficiency before and after."""
    import torch
    r = finder.result()
    nb = C.c_size_t(0)
    from paper_2505_22822_amd import _abi
    cap = int(finder.out["offsets"].numel()) - 1
    assert _abi.load().ckf_resolve_workspace_size(cap, ev.n_meas, C.byref(nb)) == 0
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=finder.out["offsets"].device)
    times = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep, rounds = ckf.resolve(finder.out, ev.n_meas, stream=stream, workspace=ws, max_rounds=max_rounds)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    keep = keep.cpu().numpy()
    before, after = track_rates(ev, r), track_rates(ev, r, keep)
    return dict(ms=round(float(np.mean(times[1:])), 4), rounds=rounds, tracks_in=int(r["n_tracks"]),
                removed=int(np.sum(keep[:r["n_tracks"]] == 0)), before=before, after=after,
                efficiency_before=round(efficiency(ev, r), 5), efficiency_after=round(efficiency(ev, kept_tracks(r, keep)), 5),
                traffic=_measured(RESOLVE_TRAFFIC, (int(r["n_tracks"]), int(r["offsets"][r["n_tracks"]]))),
                max_rounds=max_rounds,
                note="wall time of one call and its synchronisation (the rounds run on the device, unused ones "
                     "return at once); traffic: HBM bytes of its kernels (counters)")


def measure_cluster(ckf, geo, det, cells, stream, reps):
    """Clustering of the batch's cells: device time of one ckf_cluster call
    (HIP events on the launch stream around its kernels, mean of reps) and
    the HBM roofline of its algorithmic bytes: the cells read once (c0, c1,
    q: 12 B) and the row offsets (4 B), every cell's cluster index written
    (4 B), per cluster loc, var and spacepoint (28 B), the measurement
    offsets (4 B per row)."""
    import torch
    from synth.cells import cell_grid
    _, pitch = cell_grid(det)
    cl = ckf.Clusterer(geo, ckf.CellBatch.from_cells(cells), torch.as_tensor(pitch, device="cuda"))
    cl.enqueue(stream)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        cl.enqueue(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    r = cl.result()
    rows = cells.n_events * cells.n_surfaces
    algo = 16 * cells.n_cells + 28 * r["n_meas"] + 8 * rows
    measure_cluster.last = cl
    return dict(cells=cells.n_cells, clusters=r["n_meas"], status=r["status"], ms=round(ms, 4),
                cells_per_s=round(cells.n_cells / (ms * 1e-3), 1),
                roofline=dict(bound="hbm", achieved=round(algo / (ms * 1e-3) / 1e9, 1), peak=8000.0, unit="GB/s",
                              frac=round(algo / (ms * 1e-3) / 8e12, 5),
                              traffic=_measured(CLUSTER_TRAFFIC, (int(cells.n_cells), int(r["n_meas"]))), kernel="k_cl_*",
                              algorithmic_bytes=int(algo)))


SEED_LAYERS = [0, 1, 2, 3]  # the pixel barrel layers, outwards


def measure_chain(ckf, geo, fld, det, cells, evs, cl, cl_ms, stream, reps):
    """Seeding on the batch's clusters (device time of one ckf_seed, mean of
    reps), then the track finder on the clusters with those seeds (one
    call): the chain cells -> clusters -> seeds -> tracks, and the share of
    central particles (|eta| < 1.2, pT > 0.6 GeV, |z_vertex| < 150 mm) whose
    clusters make the majority of a track."""
    import torch
    r = cl.result()
    m = r["n_meas"]
    args = (geo, cells.n_events, cl.offsets, cl.spacepoints[:m], cl.loc[:m], SEED_LAYERS, 2.0)
    sd, n = ckf.seed(*args, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ckf.seed(*args, cap_seeds=int(sd["params"].shape[0]), stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    seed_ms = e0.elapsed_time(e1) / reps
    work = torch.zeros(4, dtype=torch.int64, device=cl.offsets.device)
    ckf.seed(*args, cap_seeds=int(sd["params"].shape[0]), stream=stream, counters=work)
    torch.cuda.synchronize()
    units = [int(x) for x in work.cpu()]
    seed_f64 = sum(u * f for u, f in zip(units, SEED_FLOPS))
    seed_frac = seed_f64 / PEAK_FP64 / (seed_ms * 1e-3)
    b = ckf.Batch(cells.n_events, cells.n_surfaces, cl.offsets, cl.loc[:m].contiguous(), cl.var[:m].contiguous(),
                  sd["event"].contiguous(), sd["surface"].contiguous(), sd["params"].contiguous(),
                  sd["cov"].contiguous())
    timer = ckf.KernelTimer()
    f = ckf.Finder(geo, fld, b, ckf.config(), ckf.launch(timer=timer), counters=False)
    f.enqueue(stream)
    res = f.result(check=False)
    f.enqueue(stream)
    torch.cuda.synchronize()
    find_ms = timer.elapsed_ms()
    flags = int(res["status"][0])
    # truth of a cluster: its largest-charge cell's particle (global particle ids per event)
    cc = r["cell_cluster"]
    o = np.lexsort((-cells.q, cc))
    first = o[np.r_[True, cc[o][1:] != cc[o][:-1]]]
    cell_event = np.repeat(np.arange(cells.n_events), np.diff(cells.offsets[::cells.n_surfaces]))
    part = np.full(m, -1, np.int64)
    base = np.cumsum([0] + [len(e.particle_pt) for e in evs])
    pid = cells.particle[first]
    part[cc[first]] = np.where(pid >= 0, pid + base[cell_event[first]], -1)
    tid = np.repeat(np.arange(res["n_tracks"]), np.diff(res["offsets"]))
    tp = part[res["meas"]]
    found = set()
    if res["n_tracks"]:
        key = tid.astype(np.int64) * (base[-1] + 1) + (tp + 1)
        uk, cnt = np.unique(key, return_counts=True)
        t_of, p_of = uk // (base[-1] + 1), uk % (base[-1] + 1) - 1
        n_of = np.diff(res["offsets"])[t_of]
        ok = (p_of >= 0) & (cnt > n_of / 2)
        found = set(p_of[ok].tolist())
    cen = np.concatenate([base[i] + np.nonzero((np.abs(e.particle_eta) < 1.2) & (e.particle_pt > 0.6) &
                                               (np.abs(e.particle_vtx[:, 2]) < 150))[0] for i, e in enumerate(evs)])
    eff = float(np.mean([p in found for p in cen.tolist()])) if len(cen) else 0.0
    chain_ms = cl_ms + seed_ms + find_ms
    return dict(seeds=n, seed_ms=round(seed_ms, 4), seeds_per_s=round(n / (seed_ms * 1e-3), 1),
                tracks=res["n_tracks"], find_ms=round(find_ms, 4), chain_ms=round(chain_ms, 4),
                chain_tracks_per_s=round(res["n_tracks"] / (chain_ms * 1e-3), 1), central_particles=int(len(cen)),
                central_found=round(eff, 5), find_status_flags=flags,
                seed_traffic=_measured(SEED_TRAFFIC, (int(m), int(n))),
                seed_work=dict(mt_doublets=units[0], bm_doublets=units[1], cot_comparisons=units[2],
                               triplets=units[3]),
                seed_roofline=dict(bound="alu", achieved=round(seed_frac * PEAK_FP64 / 1e12, 3),
                                   peak=PEAK_FP64 / 1e12, unit="TFLOP/s", frac=round(seed_frac, 5),
                                   fp64_flop=int(seed_f64), kernel="ckf_seed (all its kernels)"),
                note="device times of one ckf_cluster, one ckf_seed and one ckf_find (kernel timer) on the batch; "
                     "seed_traffic: HBM bytes of one ckf_seed call (counters); seed_roofline: the triplet search's "
                     "counted FP64 work (SEED_FLOPS per unit) over the call's time, against the FP64 vector peak")


def roofline_of(m, form, shape):
    c = dict(m["counters"])
    f32 = sum(c.get(k, 0) * UNIT_FLOPS[k][0] for k in UNIT_FLOPS)
    f64 = sum(c.get(k, 0) * UNIT_FLOPS[k][1] for k in UNIT_FLOPS)
    mf = c.get("mlp_blocks", 0) * MFMA_FLOP_PER_BLOCK
    t = m["kernel_ms"] * 1e-3
    frac = (f32 / PEAK_FP32 + f64 / PEAK_FP64 + mf / PEAK_BF16) / t
    key = (form, shape["grid"], shape["seeds_per_group"], shape["waves_per_simd"])
    return dict(bound="alu", achieved=round(frac * PEAK_FP32 / 1e12, 3), peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                frac=round(frac, 5), traffic=_measured(MEASURED_TRAFFIC, key),
                simt_efficiency=_measured(MEASURED_SIMT, key), code=code_hash(),
                kernel="k_ckf", kernel_ms=round(m["kernel_ms"], 4), fp32_flop=f32, fp64_flop=f64, bf16_mfma_flop=mf,
                note="achieved = FP32-equivalent rate (F32 + 2*F64 + F_bf16/15.9)/t against the FP32 vector peak")


def loop_use(c):
    """Lane use of the search's data-dependent loops: iterations summed over
    the lanes that ran the loop, over 64 times the longest lane's iterations
    summed over the wave's passes (1.0: every lane busy for every pass)."""
    out = {}
    for k in ("list", "next", "land", "win"):
        w = c.get(k + "_wave", 0)
        out[k] = round(c.get(k + "_lane", 0) / (64.0 * w), 4) if w else None
    return out


def phase_line(c, label):
    tot = max(1, c["cycles_step"])
    lu = loop_use(c)
    return ("# {} instrumented run, share of step time: phase1 (nav+leg) {:.2f}, search {:.2f}, out {:.2f}; "
            "lane-average navigation / phase1 {:.2f}, next-layer search / navigation {:.2f}; "
            "lane occupancy {:.2f}; clocks per 64-lane pass {:.0f}; loop lane use: listing {}, next layer {}, "
            "landing {}, window {}").format(
        label, c["cycles_leg"] / tot, c["cycles_search"] / tot, c["cycles_out"] / tot,
        c["cycles_nav"] / 64.0 / max(1, c["cycles_leg"]), c["cycles_next"] / max(1, c["cycles_nav"]),
        c["steps"] / 64.0 / max(1, c["chunks"]), tot / max(1, c["chunks"]), lu["list"], lu["next"], lu["land"],
        lu["win"])


CYCLE_KEYS = ("cycles_leg", "cycles_search", "cycles_out", "cycles_nav", "cycles_step", "cycles_next", "chunks",
              "list_lane", "list_wave", "next_lane", "next_wave", "land_lane", "land_wave", "win_lane", "win_wave")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=64)
    ap.add_argument("--mu", type=float, default=200.0)
    ap.add_argument("--cpu-events", type=int, default=64,
                    help="events of the batch the oracle's CPU baseline runs on (default: all 64, a few seconds on "
                         "16 host cores)")
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--seeds-per-group", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0, help="kernel register variant: waves per SIMD (1, 2 or 3; 0: the autotuner picks)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--no-learned", action="store_true", help="plain form only")
    ap.add_argument("--train-events", type=int, default=34,
                    help="mu=200 training events (seeds 5000 + i) whose plain-search tracks give the pairs "
                         "(34: about 2M pairs)")
    ap.add_argument("--heldout-events", type=int, default=8,
                    help="held-out mu=200 events (seeds 5500 + i) on which the threshold is chosen")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--min-prob", type=float, default=0.0,
                    help="learned form: summed top-3 probability above which the proposal is used (0: the "
                         "smallest of the candidates whose held-out efficiency stays within the allowance)")
    ap.add_argument("--map-events", type=int, default=16,
                    help="mu=200 events with truth integrated through the solenoid map, found in the map "
                         "(0: skip)")
    ap.add_argument("--single-thread-seeds", type=int, default=4000,
                    help="seeds of the oracle's single-thread run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_read=4 * n, copy_bytes_written=4 * n, launches=3)))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this track finder has no multi-GPU path "
              "(events would be sharded across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)
    say = lambda msg: print(msg, file=sys.stderr, flush=True)

    t0 = time.time()
    # every event set is generated before the GPU is touched (forked workers)
    evs, batch, cells = make_events([6000 + i for i in range(args.events)], args.mu, args.workers, cells=True)
    say(f"# generated {batch.n_events} events, {batch.n_seeds} seeds, {batch.n_meas} measurements, "
        f"{cells.n_cells} cells in {time.time() - t0:.1f} s")
    t0 = time.time()
    umus = uneven_mus(len(UNEVEN_SEEDS))
    uevs, ubatch = make_events(UNEVEN_SEEDS, umus, args.workers)
    useeds = np.bincount(ubatch.seed_event, minlength=ubatch.n_events)
    say(f"# uneven batch: {ubatch.n_events} events, mu {umus.min():.0f}..{umus.max():.0f}, seeds per event "
        f"{useeds.min()}..{useeds.max()} ({ubatch.n_seeds} in all), generated in {time.time() - t0:.1f} s")
    mevs = mbatch = None
    if args.map_events > 0:
        t0 = time.time()
        mevs, mbatch = make_events([6200 + i for i in range(args.map_events)], args.mu, args.workers, field_map=True)
        say(f"# field-map batch: {mbatch.n_events} events with truth integrated through the solenoid map, "
            f"{mbatch.n_seeds} seeds, generated in {time.time() - t0:.1f} s")
    tevs = hevs = None
    if not args.no_learned:
        t0 = time.time()
        _, tbatch = make_events([5000 + i for i in range(args.train_events)], args.mu, args.workers)
        hevs, hbatch = make_events([5500 + i for i in range(args.heldout_events)], args.mu, args.workers)
        say(f"# training events: {tbatch.n_events} ({tbatch.n_seeds} seeds); held-out events for the threshold: "
            f"{hbatch.n_events}; generated in {time.time() - t0:.1f} s")

    import torch
    import paper_2505_22822_amd as ckf
    from paper_2505_22822_amd import autotune
    from synth import barrel_endcap
    det = barrel_endcap()
    geo = ckf.Geometry(det.as_arrays())
    fld = ckf.UniformField(0.0, 0.0, 2.0)
    b = ckf.Batch.from_event(batch)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    fixed = bool(args.grid or args.seeds_per_group or args.waves)

    def pick(model=None):
        if fixed:
            return dict(grid=args.grid, seeds_per_group=args.seeds_per_group, waves_per_simd=args.waves)
        waves = (3, 2) if model is None else (3, 2, 1)
        shapes = [dict(grid=n_cu * 4 * w * g, seeds_per_group=s, waves_per_simd=w)
                  for w in waves for g in (1, 2) for s in (32, 48)]
        shape, _ = autotune.tune(geo, fld, b, ckf.config(), shapes=shapes, reps=2, verbose=True,
                                 use_cache=not args.retune and model is None, model=model)
        return shape

    stream = torch.cuda.Stream()
    shape_plain = pick()
    say(f"# plain launch shape {shape_plain}")
    plain = measure(ckf, geo, fld, b, shape_plain, args.steps, args.warmup, stream)
    eff_plain = efficiency(batch, plain["result"])
    say(f"# plain: {plain['tracks_per_s'] / 1e6:.2f} M tracks/s, kernel {plain['kernel_ms']:.3f} ms, "
        f"efficiency {eff_plain:.4f}")
    cyc_plain = {k: plain["counters"].pop(k) for k in CYCLE_KEYS}
    say(phase_line({**plain["counters"], **cyc_plain}, "plain"))
    e2e = measure_end_to_end(ckf, geo, fld, batch, shape_plain, stream, max(3, args.steps // 4))
    say(f"# end to end (host -> device inputs, ckf_find, device -> host outputs): {e2e['ms']:.2f} ms per batch, "
        f"{e2e['tracks_per_s'] / 1e6:.2f} M tracks/s (inputs {e2e['bytes_in'] / 1e6:.0f} MB, outputs "
        f"{e2e['bytes_out'] / 1e6:.0f} MB)")

    ub = ckf.Batch.from_event(ubatch)
    um = measure(ckf, geo, fld, ub, shape_plain, args.steps, args.warmup, stream)
    uneven = dict(events=ubatch.n_events, mu_min=round(float(umus.min()), 2), mu_max=round(float(umus.max()), 2),
                  seeds=ubatch.n_seeds, seeds_per_event_min=int(useeds.min()), seeds_per_event_max=int(useeds.max()),
                  measurements=ubatch.n_meas, tracks=um["result"]["n_tracks"],
                  plain=dict(tracks_per_s=round(um["tracks_per_s"], 1), ms_per_step=round(um["ms_per_step"], 4),
                             kernel_ms=round(um["kernel_ms"], 4), efficiency=round(efficiency(ubatch, um["result"]), 5),
                             launch=shape_plain))
    del um["counters"]
    say(f"# uneven batch, plain: {uneven['plain']['tracks_per_s'] / 1e6:.2f} M tracks/s, kernel "
        f"{uneven['plain']['kernel_ms']:.3f} ms, efficiency {uneven['plain']['efficiency']:.4f}")

    field_map = None
    if mbatch is not None:
        from synth.field import solenoid_map
        fmap = ckf.FieldMap(solenoid_map())
        mb = ckf.Batch.from_event(mbatch)
        mshape = dict(grid=n_cu * 4 * 2, seeds_per_group=48, waves_per_simd=2)
        mm = measure(ckf, geo, fmap, mb, mshape, max(3, args.steps // 4), args.warmup, stream)
        field_map = dict(events=mbatch.n_events, seeds=mbatch.n_seeds, measurements=mbatch.n_meas,
                         tracks=mm["result"]["n_tracks"], truth="integrated through the solenoid map (FP64 RK4)",
                         tracks_per_s=round(mm["tracks_per_s"], 1), ms_per_step=round(mm["ms_per_step"], 4),
                         kernel_ms=round(mm["kernel_ms"], 4), efficiency=round(efficiency(mbatch, mm["result"]), 5),
                         launch=mshape, roofline=roofline_of(mm, "map", mshape))
        say(f"# field map, plain: {field_map['tracks_per_s'] / 1e6:.2f} M tracks/s, kernel "
            f"{field_map['kernel_ms']:.3f} ms, efficiency {field_map['efficiency']:.4f} on {mbatch.n_events} events")
        del mb, mm, fmap

    c0 = plain["counters"]
    fit = measure_fit(ckf, geo, fld, b, shape_plain, stream, max(3, args.steps // 4),
                      c0["rk_trials"] / max(1, c0["legs"]))
    say(f"# fit of the plain search's {fit['tracks']} tracks ({fit['measurements']} measurements): "
        + "; ".join(f"{k} {fit[k]['tracks_per_s'] / 1e6:.2f} M tracks/s, kernel {fit[k]['kernel_ms']:.3f} ms, "
                    f"fitted {fit[k]['fitted']:.5f}" for k in ("rts", "two_filter")))
    amb = measure_resolve(ckf, fit.pop("_finder"), batch, stream)
    clu = measure_cluster(ckf, geo, det, cells, stream, max(3, args.steps // 4))
    say(f"# clustering of the batch's {clu['cells']} cells: {clu['clusters']} clusters in {clu['ms']:.3f} ms "
        f"({clu['cells_per_s'] / 1e9:.2f} G cells/s, {clu['roofline']['achieved']:.0f} GB/s algorithmic), "
        f"status {clu['status']}")
    chain = measure_chain(ckf, geo, fld, det, cells, evs, measure_cluster.last, clu["ms"], stream,
                          max(3, args.steps // 4))
    say(f"# seeding on the clusters: {chain['seeds']} seeds in {chain['seed_ms']:.3f} ms; track finding with them: "
        f"{chain['tracks']} tracks in {chain['find_ms']:.3f} ms; chain cells -> tracks {chain['chain_ms']:.2f} ms "
        f"({chain['chain_tracks_per_s'] / 1e6:.2f} M tracks/s), central particles found {chain['central_found']:.4f}; "
        f"seeding work {chain['seed_work']}, FP64 rate {chain['seed_roofline']['achieved']} TFLOP/s "
        f"({chain['seed_roofline']['frac']:.3f} of peak)")
    say(f"# ambiguity resolution of the plain search's tracks: {amb['ms']:.2f} ms, {amb['rounds']} rounds, "
        f"{amb['removed']} of {amb['tracks_in']} removed; fake rate {amb['before']['fake_rate']:.5f} -> "
        f"{amb['after']['fake_rate']:.5f}, duplicate rate {amb['before']['duplicate_rate']:.5f} -> "
        f"{amb['after']['duplicate_rate']:.5f}, efficiency {amb['efficiency_before']:.4f} -> "
        f"{amb['efficiency_after']:.4f}")

    learned_info = None
    head = plain
    if not args.no_learned:
        from paper_2505_22822_amd import learned
        tb = ckf.Batch.from_event(tbatch)
        t1 = time.time()
        params, log, info = learned.train_from_batches(geo, fld, [tb], epochs=args.epochs, batch=4096, lr=1e-3,
                                                       seed=0, stream=stream)
        torch.cuda.synchronize()
        t2 = time.time()
        say(f"# training: {info['pairs']} pairs ({info['dropped']} dropped) from {tbatch.n_events} events; "
            f"{log.steps} Adam steps in {t2 - t1:.1f} s; loss {log.loss[0]:.3f} -> "
            f"{log.loss[-1]:.3f}; validation top-1 {log.val_top1:.3f}, top-3 {log.val_top3:.3f}, "
            f"confident {log.val_confident:.3f} (of which right {log.val_confident_right:.4f})")
        del tb, tbatch
        model = ckf.Model(params)
        shape_learned = pick(model)
        say(f"# learned launch shape {shape_learned}")
        # the threshold: the smallest candidate whose efficiency on the held-out events stays within the
        # allowance of the plain form's there (chosen before the evaluation batch is looked at)
        hb = ckf.Batch.from_event(hbatch)
        h_plain = efficiency(hbatch, _find_once(ckf, geo, fld, hb, shape_plain))
        choice = []
        chosen = None
        for th in THRESHOLDS:
            e = efficiency(hbatch, _find_once(ckf, geo, fld, hb, shape_learned, model,
                                              ckf.config(learned_min_prob=th)))
            choice.append(dict(min_prob=th, efficiency=round(e, 5)))
            if chosen is None and e >= h_plain - EFF_ALLOWANCE + EFF_MARGIN:
                chosen = th
        if chosen is None:
            chosen = THRESHOLDS[-1]
        if args.min_prob > 0:
            chosen = args.min_prob
        say(f"# threshold on {hbatch.n_events} held-out events: plain efficiency {h_plain:.4f}; "
            + ", ".join(f"{c['min_prob']}: {c['efficiency']:.4f}" for c in choice) + f"; chosen {chosen}")
        del hb, hbatch

        def learned_run(th, audit):
            lm = measure(ckf, geo, fld, b, shape_learned, args.steps, args.warmup, stream, model=model,
                         audit=audit, cfg=ckf.config(learned_min_prob=th))
            eff = efficiency(batch, lm["result"])
            c = lm["counters"]
            say(f"# learned at {th}: {lm['tracks_per_s'] / 1e6:.2f} M tracks/s, kernel {lm['kernel_ms']:.3f} ms, "
                f"efficiency {eff:.4f}; network rows {c['mlp_rows']} of {c['navigations']} navigations, "
                f"proposals used {c['proposals']}, listings differing from the geometric one {c['proposal_misses']}, "
                f"seeds affected {int(lm['seed_flags'].sum()) if audit else -1}")
            return lm, eff

        lm, eff_learned = learned_run(chosen, True)
        c = lm["counters"]
        cyc_learned = {k: lm["counters"].pop(k) for k in CYCLE_KEYS}
        say(phase_line({**lm["counters"], **cyc_learned}, "learned"))
        at_cfg = None
        if abs(chosen - CFG_MIN_PROB) > 1e-12:
            l95, e95 = learned_run(CFG_MIN_PROB, False)
            at_cfg = dict(min_prob=CFG_MIN_PROB, tracks_per_s=round(l95["tracks_per_s"], 1),
                          ms_per_step=round(l95["ms_per_step"], 4), kernel_ms=round(l95["kernel_ms"], 4),
                          efficiency=round(e95, 5), equal_efficiency=bool(e95 >= eff_plain - EFF_ALLOWANCE),
                          proposals=l95["counters"]["proposals"])
            del l95
        lu = measure(ckf, geo, fld, ub, shape_learned, args.steps, args.warmup, stream, model=model,
                     cfg=ckf.config(learned_min_prob=chosen))
        uneven["learned"] = dict(min_prob=chosen, tracks_per_s=round(lu["tracks_per_s"], 1),
                                 ms_per_step=round(lu["ms_per_step"], 4), kernel_ms=round(lu["kernel_ms"], 4),
                                 efficiency=round(efficiency(ubatch, lu["result"]), 5), launch=shape_learned)
        del lu
        learned_info = dict(tracks_per_s=round(lm["tracks_per_s"], 1), ms_per_step=round(lm["ms_per_step"], 4),
                            kernel_ms=round(lm["kernel_ms"], 4), min_prob=chosen,
                            threshold_choice=dict(events=args.heldout_events, plain_efficiency=round(h_plain, 5),
                                                  allowance=EFF_ALLOWANCE, margin=EFF_MARGIN, candidates=choice),
                            efficiency=round(eff_learned, 5), launch=shape_learned,
                            proposals=c["proposals"], network_rows=c["mlp_rows"], navigations=c["navigations"],
                            listing_misses=c["proposal_misses"], seeds_affected=int(lm["seed_flags"].sum()),
                            at_configured_threshold=at_cfg,
                            training=dict(events=args.train_events, pairs=info["pairs"], dropped=info["dropped"],
                                          epochs=log.epochs, adam_steps=log.steps, seconds=round(t2 - t1, 2),
                                          loss_first=round(log.loss[0], 4), loss_last=round(log.loss[-1], 4),
                                          val_top1=round(log.val_top1, 4), val_top3=round(log.val_top3, 4),
                                          val_confident=round(log.val_confident, 4)),
                            counters=c)
        head = lm

    cpu = None
    if args.cpu_events > 0:
        cpu = cpu_baseline(batch, min(args.cpu_events, batch.n_events))
        cpu["single_thread"] = cpu_single_thread(batch, args.single_thread_seeds)
    form = "learned proposal" if learned_info else "plain"
    line = dict(metric="CKF tracks/s at mu=200 on 1 GPU; learned-proposal vs plain at equal efficiency",
                value=round(head["tracks_per_s"], 1), unit="tracks/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(head["ms_per_step"], 4), higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32+f64" + ("+bf16" if learned_info else ""),
                data="synthetic",
                config=dict(workload=f"{batch.n_events} x mu={args.mu:g} events, barrel+endcap, 1% X0, 2 T, "
                                     f"{form} CKF, one hipGraph-captured ckf_find per step",
                            events=batch.n_events, seeds=batch.n_seeds, measurements=batch.n_meas,
                            tracks=head["result"]["n_tracks"],
                            launch=learned_info["launch"] if learned_info else shape_plain),
                plain=dict(tracks_per_s=round(plain["tracks_per_s"], 1), ms_per_step=round(plain["ms_per_step"], 4),
                           kernel_ms=round(plain["kernel_ms"], 4), efficiency=round(eff_plain, 5), launch=shape_plain),
                learned=learned_info,
                equal_efficiency=(learned_info["efficiency"] >= eff_plain - EFF_ALLOWANCE) if learned_info else None,
                learned_faster=(learned_info["tracks_per_s"] > plain["tracks_per_s"]) if learned_info else None,
                roofline=roofline_of(head, "learned" if learned_info else "plain",
                                     learned_info["launch"] if learned_info else shape_plain),
                plain_roofline=roofline_of(plain, "plain", shape_plain),
                end_to_end=e2e, uneven=uneven, field_map=field_map,
                fit=fit, ambiguity=amb, clustering=clu, chain=chain, cpu_baseline=cpu, counters=plain["counters"],
                clocks=cyc_plain, loop_lane_use=loop_use(cyc_plain))
    print(json.dumps(line))


if __name__ == "__main__":
    main()
