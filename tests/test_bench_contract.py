"""The benchmark's host-side contract (no GPU needed): it refuses more than
one GPU with a message, and its roofline object is self-consistent (frac =
achieved / peak, inversely proportional to the kernel time, measured traffic
reported only for the launch shapes and the library sources it was
measured on)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_roofline_object_is_self_consistent():
    sys.path.insert(0, ROOT)
    import bench
    counters = {k: 1000 * (i + 1) for i, k in enumerate(bench.UNIT_FLOPS)}
    counters["mlp_blocks"] = 77
    shape = dict(grid=3072, seeds_per_group=48, waves_per_simd=3)
    a = bench.roofline_of(dict(counters=counters, kernel_ms=2.0), "plain", shape)
    b = bench.roofline_of(dict(counters=counters, kernel_ms=4.0), "plain", shape)
    assert a["bound"] == "alu" and a["unit"] == "TFLOP/s" and a["peak"] == 157.3
    assert abs(a["frac"] - a["achieved"] / a["peak"]) <= 1e-5 * max(1.0, a["frac"])
    assert abs(a["frac"] - 2.0 * b["frac"]) <= 2e-5 * max(1.0, a["frac"])
    assert a["fp32_flop"] > 0 and a["fp64_flop"] > 0 and a["bf16_mfma_flop"] == 77 * bench.MFMA_FLOP_PER_BLOCK
    key = ("plain", 3072, 48, 3)
    saved = dict(bench.MEASURED_TRAFFIC), dict(bench.MEASURED_SIMT)
    try:
        bench.MEASURED_TRAFFIC[key] = (1.5e9, bench.code_hash())
        bench.MEASURED_SIMT[key] = (0.5, bench.code_hash())
        a = bench.roofline_of(dict(counters=counters, kernel_ms=2.0), "plain", shape)
        assert a["traffic"] == 1.5e9 and a["simt_efficiency"] == 0.5 and a["code"] == bench.code_hash()
        other = bench.roofline_of(dict(counters=counters, kernel_ms=2.0), "plain",
                                  dict(grid=1234, seeds_per_group=16, waves_per_simd=1))
        assert other["traffic"] is None and other["simt_efficiency"] is None
        # values measured on other sources are not reported
        bench.MEASURED_TRAFFIC[key] = (1.5e9, "0" * 16)
        bench.MEASURED_SIMT[key] = (0.5, "0" * 16)
        stale = bench.roofline_of(dict(counters=counters, kernel_ms=2.0), "plain", shape)
        assert stale["traffic"] is None and stale["simt_efficiency"] is None
    finally:
        bench.MEASURED_TRAFFIC.clear()
        bench.MEASURED_TRAFFIC.update(saved[0])
        bench.MEASURED_SIMT.clear()
        bench.MEASURED_SIMT.update(saved[1])
