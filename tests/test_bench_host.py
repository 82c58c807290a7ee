"""Host-side logic of bench.py (CPU): the source hash that ties the committed
counter summary to the kernels it measured, and the arithmetic that turns two
rocprofv3 counter runs into HBM bytes per step launch."""
import csv
import os

import pytest

import bench


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2302_04741_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = csrc / "lbm_kernels.h"
    src.write_text("// a kernel\nint f(int x) { return x + 1; }  /* one */\n")
    host = csrc / "lbm_api.hip"
    host.write_text("int g(void) { return 0; }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    src.write_text("// the same kernel, reworded\n\nint f(int x) { return x + 1; }\n"
                   "/* a block\n   comment */\n")
    assert bench.kernel_source_hash() == h0
    host.write_text("int g(void) { return 1; }\n")  # host code: not the measured kernel
    assert bench.kernel_source_hash() == h0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h0


def _write_pmc(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_counter_summary_scales_by_the_copy(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled so that the
    2 GiB copy of the same run reads and writes exactly 2 GiB; the step's bytes
    are then compared with the algorithmic 2 * 39 * 4 B per cell of 256^3."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_2302_04741_amd" / "csrc").mkdir(parents=True)  # hashed (empty)
    alg = 2 * 39 * 4 * 256 ** 3
    kib = (1 << 31) / 1024.0
    # the fetch counter reads half of the true bytes, the write counter all of them
    _write_pmc(tmp_path / "f.csv", "FETCH_SIZE",
               [("__amd_rocclr_copyBuffer", 1 << 20, kib / 2),
                ("void lbm::step_kernel<1, float, 3, 4>(...)", 1 << 24, alg / 2 / 1024 / 2),
                ("void lbm::step_kernel<1, float, 3, 4>(...)", 1 << 24, alg / 2 / 1024 / 2),
                ("void lbm::moments_kernel<1>(...)", 1 << 20, 5.0)])
    _write_pmc(tmp_path / "w.csv", "WRITE_SIZE",
               [("__amd_rocclr_copyBuffer", 1 << 20, kib),
                ("void lbm::step_kernel<1, float, 3, 4>(...)", 1 << 24, alg / 2 / 1024 * 1.01)])
    out = bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                              str(tmp_path / "summary.txt"))
    assert out["fetch_scale_from_copy"] == pytest.approx(2.0)
    assert out["write_scale_from_copy"] == pytest.approx(1.0)
    assert out["read_over_algorithmic"] == pytest.approx(1.0)
    assert out["write_over_algorithmic"] == pytest.approx(1.01)
    assert out["hbm_bytes_per_launch"] == pytest.approx(alg * 1.005, rel=1e-9)
    assert out["dispatches_averaged"] == "2 fetch, 1 write"
    assert os.path.exists(tmp_path / "summary.txt")


def test_committed_summary_is_read_back():
    """measured_traffic() returns the committed summary's bytes exactly when its
    hash matches the current sources (None otherwise); either way it never
    raises."""
    v = bench.measured_traffic()
    assert v is None or v > 0


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err
