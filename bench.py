#!/usr/bin/env python3
"""Throughput of the fused D3Q39 force-collide-stream step on one MI355X.

Workload (default): D3Q39, FP32 storage of the deviations f~_i - w_i, 256^3
periodic grid, Kolmogorov force g_x = 1e-5 sin(2 pi z/256), rho = 1,
theta = 1 + 0.05 sin(2 pi y/256), seeded random-phase velocity perturbation of
RMS 1e-3 per component, tau-hat = 0.8, 3rd-order Hermite equilibrium, full
force term (a3_F and sigma).  Inputs are synthetic and resident in HBM before
the timed region.

One "step" is one launch of the fused kernel over the whole grid.  The timed
region is exactly --steps steps, bracketed by stream synchronisation; its HIP
events are recorded on the stream the kernel runs on.  Prints one JSON line.

Roofline: the step is bound by HBM bandwidth.  Algorithmic traffic per lattice
update is one read and one write of every population, 2 * Q * s = 312 bytes
(Q = 39, s = 4 bytes); the force profile and the launch arguments add nothing
per cell.  `traffic` is the measured HBM traffic per launch from the committed
rocprofv3 counter summary, valid only while the kernel sources are unchanged.

CPU baseline: the FP64 CPU oracle (as it stands) on the same workload at full
size for a bounded number of steps, on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
PMC_SUMMARY = os.path.join(ROOT, "profiles", "step_d3q39_f32_256cube_pmc.txt")


def kernel_source_hash() -> str:
    """Hash of the HIP sources that make up the step kernel."""
    csrc = os.path.join(ROOT, "paper_2302_04741_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; else None."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    vals = {}
    with open(PMC_SUMMARY) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _pmc_per_kernel(csv_path, counter):
    import csv
    import collections

    vals = collections.defaultdict(list)
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                vals[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return vals


def summarize_pmc(fetch_csv: str, write_csv: str, out_path: str) -> dict:
    """Turn two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch)
    into HBM bytes per step launch.  Each counter is scaled by what it reads for
    the plain 2 GiB device copy (--copy-calib) of the same run: a copy moves
    exactly 2 GiB in each direction."""
    fetch = _pmc_per_kernel(fetch_csv, "FETCH_SIZE")
    write = _pmc_per_kernel(write_csv, "WRITE_SIZE")
    copy_bytes = float(1 << 31)

    def pick(vals, needle, big=True):
        keys = [k for k in vals if needle in k[0]]
        if big:
            keys = [max(keys, key=lambda k: k[1])]
        v = [x for k in keys for x in vals[k]]
        return sum(v) / len(v), len(v)

    f_copy, _ = pick(fetch, "copyBuffer")
    w_copy, _ = pick(write, "copyBuffer")
    f_step, nf = pick(fetch, "step_kernel")
    w_step, nw = pick(write, "step_kernel")
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    read_b = f_step * 1024.0 * f_scale
    write_b = w_step * 1024.0 * w_scale
    alg = 2 * 39 * 4 * 256 ** 3
    out = {
        "kernel_source_hash": kernel_source_hash(),
        "fetch_kib_per_launch_raw": round(f_step, 1),
        "write_kib_per_launch_raw": round(w_step, 1),
        "fetch_scale_from_copy": round(f_scale, 4),
        "write_scale_from_copy": round(w_scale, 4),
        "hbm_read_bytes_per_launch": round(read_b),
        "hbm_write_bytes_per_launch": round(write_b),
        "hbm_bytes_per_launch": round(read_b + write_b),
        "algorithmic_bytes_per_launch": alg,
        "traffic_over_algorithmic": round((read_b + write_b) / alg, 4),
        "read_over_algorithmic": round(read_b / (alg / 2), 4),
        "write_over_algorithmic": round(write_b / (alg / 2), 4),
        "dispatches_averaged": "%d fetch, %d write" % (nf, nw),
    }
    with open(out_path, "w") as fh:
        fh.write("# HBM traffic of the fused step kernel, D3Q39 FP32 (deviation storage), 256^3 Kolmogorov\n")
        fh.write("# counter runs (repo root, MI355X), one counter per run:\n")
        fh.write("#   rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_fetch -o pmc -- python3 bench.py "
                 "--steps 5 --warmup 2 --cpu-steps 0 --copy-calib\n")
        fh.write("#   rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_write -o pmc -- python3 bench.py "
                 "--steps 5 --warmup 2 --cpu-steps 0 --copy-calib\n")
        fh.write("# summarised by:\n#   python3 bench.py --summarize-pmc "
                 "gpurun_out/pmc_fetch/pmc_counter_collection.csv "
                 "gpurun_out/pmc_write/pmc_counter_collection.csv\n")
        fh.write("# scale = 2 GiB / counter value of the 2 GiB plain device copy in the same run\n")
        for k, v in out.items():
            fh.write("%s: %s\n" % (k, v))
    return out


def cpu_baseline(wl, steps: int):
    import oracle

    g = wl.force_field()
    sim = oracle.OracleSim(1, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta, g,
                           force_order=wl.force_order)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    return {"value": wl.ncell * steps / dt / 1e6, "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle, full %dx%dx%d grid of the same workload, %d steps "
                      "(%.1f s, init excluded)" % (*wl.dims, steps, dt)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid side (default 256)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16dev"])
    ap.add_argument("--block", type=int, default=0, help="threads per block (0 = default)")
    ap.add_argument("--cpu-steps", type=int, default=6,
                    help="oracle steps of the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter summary under profiles/ and exit (no GPU)")
    args = ap.parse_args(argv)

    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1],
                                       PMC_SUMMARY)))
        return 0

    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path is the single-GPU fused step "
              "(multi-GPU slab decomposition is a design, not built); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch

    from paper_2302_04741_amd import sim as lbm_sim
    from paper_2302_04741_amd import workloads

    wl = workloads.kolmogorov_3d(n=args.n)
    s = lbm_sim.from_workload(wl, storage=args.storage)
    if args.block:
        s.set_block(args.block)
    stream = s.stream
    torch.cuda.synchronize()

    s.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    s.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_events = ev0.elapsed_time(ev1)
    rho, u, th = s.moments()
    finite = bool(torch.isfinite(u).all().item() and torch.isfinite(th).all().item())
    if not finite:
        print("non-finite fields after the run", file=sys.stderr)
        return 1

    if args.copy_calib:
        a = torch.empty(1 << 29, dtype=torch.float32, device="cuda")  # 2 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    N = wl.ncell
    Q = 39
    sbytes = {"f32": 4, "f64": 8, "f16dev": 2}[args.storage]
    ms_per_step = ms_events / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    bytes_per_launch = 2.0 * Q * sbytes * N
    achieved = bytes_per_launch / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic() if (args.n == 256 and args.storage == "f32") else None

    out = {
        "metric": "D3Q39 force-collide-stream MLUPS",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f16dev": "f16 storage, f32 arithmetic"}[args.storage],
        "data": "synthetic",
        "config": {
            "workload": "D3Q39 %d^3 periodic Kolmogorov flow, %s deviation storage, tau=0.8, "
                        "3rd-order equilibrium, force with a3_F and sigma"
                        % (args.n, args.storage.upper()),
            "grid": [args.n] * 3,
            "storage": args.storage,
            "block": args.block or "default",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "wall_s_timed_region": round(wall, 4),
    }
    if args.cpu_steps > 0:
        del s, rho, u, th
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
