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
                         "--cpu-steps", "0"])
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
