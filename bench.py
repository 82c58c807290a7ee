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
    ap.add_argument("--storage", default="f32", choices=["f32", "f64"])
    ap.add_argument("--block", type=int, default=0, help="threads per block (0 = default)")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="oracle steps of the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args(argv)

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
    sbytes = 4 if args.storage == "f32" else 8
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
        "dtype": "f32" if args.storage == "f32" else "f64",
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
