"""The benchmark's output contract on the GPU: one JSON line with the metric,
the roofline of the dominant kernel (measured live), the access-pattern
ceiling and the repeats, from a short run on a small grid."""
import contextlib
import io
import json

import pytest

import bench

pytestmark = pytest.mark.gpu


def test_bench_line_fields():
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        rc = bench.main(["--n", "64", "--steps", "5", "--warmup", "2", "--repeats", "2",
                         "--cpu-steps", "0", "--no-serve"])
    assert rc == 0
    lines = [ln for ln in buf.getvalue().splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 2
    assert d["unit"] == "MLUPS" and d["value"] > 0 and d["dtype"] == "f32"
    assert "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] > 0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert r["traffic"] is None  # the counter summary is for the 256^3 grid only
    p = d["pattern_ceiling"]
    assert p["achieved"] > 0 and set(p["by_block"]) == {"256", "512", "1024"}
    assert d["repeats"]["count"] == 2


def test_bench_line_serving_fields():
    """The default line carries the serving figures (here on a short stream)."""
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        rc = bench.main(["--n", "64", "--steps", "3", "--warmup", "1", "--repeats", "0",
                         "--cpu-steps", "0", "--serve-count", "12", "--req-steps", "100",
                         "--rate", "100"])
    assert rc == 0
    lines = [ln for ln in buf.getvalue().splitlines() if ln.startswith("{")]
    d = json.loads(lines[-1])
    sv = d["serving"]
    assert sv["requests"] == 12 and sv["failed"] == 0 and sv["queued_failed"] == 0
    assert 0 < sv["p50_latency_s"] <= sv["p99_latency_s"]
    for k in ("live_aggregate_mlups", "queued_aggregate_mlups", "sequential_aggregate_mlups"):
        assert sv[k] > 0, k
    assert sv["workload"].startswith("12 D2Q37 requests")


def test_bench_line_d2q37():
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        rc = bench.main(["--lattice", "D2Q37", "--n", "256", "--storage", "f64", "--steps", "5",
                         "--warmup", "2", "--repeats", "1", "--cpu-steps", "1"])
    assert rc == 0
    lines = [ln for ln in buf.getvalue().splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert d["metric"] == "D2Q37 force-collide-stream MLUPS" and d["value"] > 0
    assert d["config"]["grid"] == [256, 256, 1] and d["dtype"] == "f64"
    assert d["config"]["workload"].startswith("D2Q37 256^2")
    r = d["roofline"]
    # 2 * 37 * 8 bytes per update
    assert abs(r["achieved"] - 592 * d["value"] / 1e3) < 1e-3 * r["achieved"] + 0.2
    assert r["traffic"] is None
    assert d["cpu_baseline"]["kind"] == "oracle" and d["cpu_baseline"]["value"] > 0
    assert "256x256x1" in d["cpu_baseline"]["single_thread"]["sample"]


@pytest.mark.parametrize("storage,floor", [("f32", 0.90), ("f16dev", 0.85)])
def test_step_stays_near_its_pattern_ceiling(storage, floor):
    """Performance guard, relative to the same machine: the fused step on the
    256^3 benchmark grid moves its bytes at least `floor` times as fast as its
    own loads and stores do without the arithmetic (best block size), so a
    change that slows the kernel fails here whatever the machine's absolute speed.
    Measured: FP32 1.02-1.03, F16 0.94-0.98."""
    import torch

    from paper_2302_04741_amd import sim, workloads

    wl = workloads.kolmogorov_3d(n=256)
    s = sim.from_workload(wl, storage=storage, stream=torch.cuda.current_stream())
    st = torch.cuda.current_stream()

    def per_call(f, n=30):
        f(3)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            f(n)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n
            best = ms if best is None else min(best, ms)
        return best

    step = per_call(s.step)
    pattern = None
    for blk in (256, 512, 1024):
        s.set_block(blk)
        t = per_call(s.pattern_pass)
        pattern = t if pattern is None else min(pattern, t)
    s.set_block(0)
    s.close()
    ratio = pattern / step  # bytes per step are the same for both
    print("%s: step %.4f ms, best bare pattern %.4f ms, ratio %.3f" % (storage, step, pattern,
                                                                        ratio), flush=True)
    assert ratio >= floor
