"""Throughput of CKF track finding on one MI355X.

Workload: a batch of 64 synthetic mu = 200 events (about 10k seeds and 80k
measurements each) in the barrel + endcap detector with 1 % X0 per module
and a uniform 2 T field, found in one persistent launch.  A step is one
ckf_find over the whole batch with inputs already resident in HBM.

Prints one JSON line: tracks/s (output tracks / device time), the roofline
object of the dominant kernel (k_ckf: algorithmic FP32 + FP64 work from the
kernel's own work-unit counters, over its average duration measured with
HIP events on its stream), and the oracle timed on the host's cores on a
bounded sample of the same events.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit counted by the kernel (FP32 flop, FP64 flop);
# the derivation is in the design doc.
UNIT_FLOPS = {
    "rk_trials": (505, 0),      # RKN4 stage algebra + 3 tangent columns + landing prediction
    "legs": (300, 400),         # bound->free, free->bound Jacobian (FP32); J C J^T (FP64)
    "navigations": (300, 0),    # helix set-up and envelope crossings
    "nav_modules": (60, 0),     # listing test of one candidate module
    "chi2_evals": (0, 15),      # 2x2 innovation chi2
    "kf_updates": (0, 450),     # gain + Joseph update
    "ms_updates": (40, 4),      # Highland width (FP32), covariance increment (FP64)
}
PEAK_FP32 = 157.3e12  # MI355X vector FP32, FLOP/s
PEAK_FP64 = 78.6e12   # MI355X vector FP64, FLOP/s


def _gen(args):
    from synth import barrel_endcap, make_event
    seed, mu = args
    return make_event(barrel_endcap(), seed, mu=mu)


def make_workload(n_events, mu, workers):
    from synth import concat_events
    jobs = [(6000 + i, mu) for i in range(n_events)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            evs = pool.map(_gen, jobs)
    else:
        evs = [_gen(j) for j in jobs]
    return evs, concat_events(evs)


def cpu_baseline(evs, batch, n_events):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=64)
    ap.add_argument("--mu", type=float, default=200.0)
    ap.add_argument("--cpu-events", type=int, default=8)
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--seeds-per-group", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0, help="kernel register variant: waves per SIMD (1 or 2)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
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
              "(events would be sharded across GPUs with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    t0 = time.time()
    evs, batch = make_workload(args.events, args.mu, args.workers)
    print(f"# generated {batch.n_events} events, {batch.n_seeds} seeds, {batch.n_meas} measurements "
          f"in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    import torch
    import paper_2505_22822_amd as ckf
    from synth import barrel_endcap
    det = barrel_endcap()
    geo = ckf.Geometry(det.as_arrays())
    fld = ckf.UniformField(0.0, 0.0, 2.0)
    b = ckf.Batch.from_event(batch)
    # launch shape: autotuned on this batch (cached per device/geometry/size/config)
    from paper_2505_22822_amd import autotune
    if args.grid or args.seeds_per_group or args.waves:
        shape = dict(grid=args.grid, seeds_per_group=args.seeds_per_group, waves_per_simd=args.waves)
    else:
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        shapes = [dict(grid=n_cu * g, seeds_per_group=s, waves_per_simd=2) for g in (8, 16) for s in (24, 32, 48)]
        shape, table = autotune.tune(geo, fld, b, ckf.config(), shapes=shapes, reps=2, verbose=True,
                                     use_cache=not args.retune)
    print(f"# launch shape {shape}", file=sys.stderr, flush=True)
    lc = lambda timer=None: ckf.launch(shape["grid"], shape["seeds_per_group"], 0, timer, shape["waves_per_simd"])

    stream = torch.cuda.Stream()
    # one run of the instrumented kernel variant counts the work units of the
    # batch (the search is deterministic, so every run does the same work)
    counting = ckf.Finder(geo, fld, b, ckf.config(), lc(), counters=True)
    counting.enqueue(stream)
    rc = counting.result()
    counters = rc["counters"]
    del counting
    # the kernel's own duration: HIP events the library records around it
    timer = ckf.KernelTimer()
    eager = ckf.Finder(geo, fld, b, ckf.config(), lc(timer), counters=False)
    kernel_ms = []
    for i in range(args.warmup + args.steps):
        eager.enqueue(stream)
        ms = timer.elapsed_ms()
        if i >= args.warmup:
            kernel_ms.append(ms)
    r = eager.result()
    n_tracks = r["n_tracks"]
    assert n_tracks == rc["n_tracks"] and np.array_equal(r["meas"], rc["meas"]), "variants disagree"
    del eager
    # the timed region: the hipGraph-captured ckf_find, replayed
    finder = ckf.Finder(geo, fld, b, ckf.config(), lc(), counters=False)
    finder.capture(stream)
    for _ in range(args.warmup):
        finder.launch_graph(stream)
    stream.synchronize()
    print(f"# warm-up done: {n_tracks} tracks", file=sys.stderr, flush=True)
    t_start, t_stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        finder.launch_graph(stream)
    t_stop.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_stop)
    rg = finder.result()
    assert rg["n_tracks"] == n_tracks and np.array_equal(rg["meas"], r["meas"]), "graph replay disagrees"
    ms_per_step = total_ms / args.steps
    value = n_tracks / (ms_per_step * 1e-3)

    cyc = {k: counters.pop(k) for k in ("cycles_leg", "cycles_search", "cycles_out", "cycles_nav", "cycles_step")}
    tot = max(1, cyc["cycles_step"])
    print("# instrumented run, share of step time: phase1 (nav+leg) {:.2f}, search {:.2f}, out {:.2f}; "
          "lane-average navigation time / phase1 {:.2f}".format(
              cyc["cycles_leg"] / tot, cyc["cycles_search"] / tot, cyc["cycles_out"] / tot,
              cyc["cycles_nav"] / 64.0 / max(1, cyc["cycles_leg"])), file=sys.stderr, flush=True)
    f32 = sum(counters[k] * UNIT_FLOPS[k][0] for k in UNIT_FLOPS)
    f64 = sum(counters[k] * UNIT_FLOPS[k][1] for k in UNIT_FLOPS)
    k_ms = float(np.mean(kernel_ms))
    t = k_ms * 1e-3
    frac = (f32 / PEAK_FP32 + f64 / PEAK_FP64) / t
    roofline = dict(bound="alu", achieved=round(frac * PEAK_FP32 / 1e12, 3), peak=PEAK_FP32 / 1e12,
                    unit="TFLOP/s", frac=round(frac, 5), traffic=None,
                    kernel="k_ckf", kernel_ms=round(k_ms, 4), fp32_flop=f32, fp64_flop=f64,
                    note="achieved = FP32-equivalent rate (F32 + 2*F64)/t against the FP32 vector peak")
    cpu = None
    if args.cpu_events > 0:
        cpu = cpu_baseline(evs, batch, min(args.cpu_events, batch.n_events))
    line = dict(metric="CKF tracks/s at mu=200 on 1 GPU", value=round(value, 1), unit="tracks/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32+f64", data="synthetic",
                config=dict(workload=f"{batch.n_events} x mu={args.mu:g} events, barrel+endcap, 1% X0, 2 T, "
                                     f"plain CKF, one hipGraph-captured ckf_find per step",
                            events=batch.n_events, seeds=batch.n_seeds, measurements=batch.n_meas,
                            tracks=n_tracks, launch=shape),
                roofline=roofline, cpu_baseline=cpu, counters=counters)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
