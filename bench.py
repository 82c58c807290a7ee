#!/usr/bin/env python3
"""Throughput of the fused D3Q39 force-collide-stream step on one MI355X.

Workload (default): D3Q39, FP32 storage of the deviations f~_i - w_i, 256^3
periodic grid, Kolmogorov force g_x = 1e-5 sin(2 pi z/256), rho = 1,
theta = 1 + 0.05 sin(2 pi y/256), seeded random-phase velocity perturbation of
RMS 1e-3 per component, tau-hat = 0.8, 3rd-order Hermite equilibrium, full
force term (a3_F and sigma).  Inputs are synthetic and resident in HBM before
the timed region.  `--lattice D2Q37` times the D2Q37 step instead, on the n^2
thermal shear wave (dtheta 0.1, Ma 0.2, transverse g = 1e-5, 4th-order
equilibrium).

One "step" is one launch of the fused kernel over the whole grid.  The timed
region is exactly --steps steps, bracketed by stream synchronisation; its HIP
events are recorded on the stream the kernel runs on.  Prints one JSON line.

Roofline: the step is bound by HBM bandwidth.  Algorithmic traffic per lattice
update is one read and one write of every population, 2 * Q * s = 312 bytes
(Q = 39, s = 4 bytes); the force profile and the launch arguments add nothing
per cell.  `traffic` is the measured HBM traffic per launch from the committed
rocprofv3 counter summary, valid only while the kernel sources are unchanged.

Serving (the latency half of the metric, `serving` in the same line): the
stream of 256 D2Q37 FP32 requests (Poisson arrivals at 20/s, L ~ U{64..1024},
2000 steps each) served by continuous batching under a 1 GiB HBM budget: p50
and p99 completion latency of the real-time run, and the aggregate MLUPS of the
real-time run, of a run with every request queued at t = 0 and of the same
requests solved one after another with the single-grid kernel.

CPU baseline: the FP64 CPU oracle (as it stands) on the same workload at full
size for a bounded number of steps, on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
# block sizes at which the bare access pattern is timed
PATTERN_BLOCKS = (256, 512, 1024)
# the arithmetic type of each storage form (F16 deviations are computed in FP32)
ARITH = {"f32": "f32", "f64": "f64", "f16dev": "f16 storage, f32 arithmetic"}
PMC_SUMMARY = os.path.join(ROOT, "profiles", "step_d3q39_f32_256cube_pmc.txt")


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


# the sources the D3Q39 FP32 step kernel is compiled from (its translation unit
# and every header it includes); host code and the other kernels' units are not
# part of it
STEP_KERNEL_SOURCES = ("fastdiv.h", "lattice_tables.h", "lbm_internal.h", "lbm_kernels.h",
                       "lbm_launch.h", "step_d3q39_f32.hip")


def kernel_source_hash() -> str:
    """Hash of the sources of the measured step kernel, comments and blank
    lines left out (an edit of a comment does not change what was measured)."""
    csrc = os.path.join(ROOT, "paper_2302_04741_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name in STEP_KERNEL_SOURCES:
            with open(os.path.join(csrc, name), encoding="utf-8") as fh:
                code = _COMMENT.sub("", fh.read())
            lines = [ln.rstrip() for ln in code.splitlines() if ln.strip()]
            h.update(name.encode())
            h.update("\n".join(lines).encode())
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
    # the counter runs wrote their CSV files as <dir>/pmc_counter_collection.csv
    dirs = [os.path.relpath(os.path.dirname(os.path.abspath(p)), ROOT)
            for p in (fetch_csv, write_csv)]
    with open(out_path, "w") as fh:
        fh.write("# HBM traffic of the fused step kernel, D3Q39 FP32 (deviation storage), 256^3 Kolmogorov\n")
        fh.write("# counter runs (repo root, MI355X), one counter per run:\n")
        for counter, d in zip(("FETCH_SIZE", "WRITE_SIZE"), dirs):
            fh.write("#   rocprofv3 --pmc %s -f csv -d %s -o pmc -- python3 bench.py "
                     "--steps 5 --warmup 2 --cpu-steps 0 --repeats 0 --copy-calib --no-serve\n"
                     % (counter, d))
        fh.write("# summarised by:\n#   python3 bench.py --summarize-pmc %s %s\n"
                 % tuple(os.path.relpath(os.path.abspath(p), ROOT) for p in (fetch_csv, write_csv)))
        fh.write("# scale = 2 GiB / counter value of the 2 GiB plain device copy in the same run\n")
        for k, v in out.items():
            fh.write("%s: %s\n" % (k, v))
    return out


def _oracle_rate(wl, steps: int, nthreads: int = 0):
    import oracle

    lat = {"D2Q37": 0, "D3Q39": 1}[wl.lattice]
    sim = oracle.OracleSim(lat, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta, wl.force_field(),
                           force_order=wl.force_order, nthreads=nthreads)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    return wl.ncell * steps / dt / 1e6, dt


def cpu_baseline(wl, steps: int):
    import oracle

    from paper_2302_04741_amd import workloads

    v, dt = _oracle_rate(wl, steps)
    cores = oracle.num_threads()
    # one host thread, on a small grid of the same workload (a bounded sample:
    # 64^3 or 256^2); the thread count is process-wide, so it is restored afterwards
    if wl.lattice == "D3Q39":
        small = workloads.kolmogorov_3d(n=64, tau_hat=wl.tau_hat)
    else:
        small = workloads.thermal_shear_2d(n=256, tau_hat=wl.tau_hat)
    v1, dt1 = _oracle_rate(small, 2, nthreads=1)
    oracle.num_threads(cores)
    return {"value": v, "unit": "MLUPS",
            "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, full %dx%dx%d grid of the same workload, %d steps "
                      "(%.1f s, init excluded), %s" % (*wl.dims, steps, dt, _cpu_model()),
            "single_thread": {"value": round(v1, 3), "unit": "MLUPS",
                              "sample": "FP64 oracle, one thread, %s grid of the same "
                                        "workload, 2 steps (%.1f s)"
                                        % ("x".join(map(str, small.dims)), dt1)}}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _grid_mix(kind: str, count: int, seed: int):
    """Workloads of a batch measurement: `serve` takes the grids, forces and
    fields of the first `count` requests of the serving stream (D2Q37,
    L ~ U{64..1024}); `small` draws `count` D2Q37 grids with L ~ U{32..256}
    from the same recipe."""
    from paper_2302_04741_amd import serve

    if kind == "serve":
        reqs = serve.make_requests(n=count, seed=seed)
    else:
        reqs = serve.make_requests(n=count, seed=seed, lmin=32, lmax=256)
    return [r.workload for r in reqs]


def bench_batch(args) -> dict:
    """Aggregate MLUPS of a mix of independent D2Q37 FP32 grids: every grid
    stepped alone with the single-grid kernel, one after another (sequential),
    against all of them advanced together by the persistent multi-grid kernel
    (one launch per step), eager and replayed from a captured graph."""
    import torch

    from paper_2302_04741_amd import sim as lbm_sim

    wls = _grid_mix(args.mix, args.count, args.seed)
    # a stream of its own: graph capture cannot run on the legacy default stream
    stream = torch.cuda.Stream()
    sims = [lbm_sim.from_workload(wl, storage=args.storage, stream=stream) for wl in wls]
    cells = sum(wl.ncell for wl in wls)
    torch.cuda.synchronize()

    def timed(fn):
        fn(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def sequential(n):
        for s in sims:
            s.step(n)

    ms_seq = timed(sequential)
    b = lbm_sim.Batch(len(sims), stream=stream)
    b.set(sims)
    if args.batch_threads or args.batch_blocks:
        b.set_launch(args.batch_threads, args.batch_blocks)
    ms_batch = timed(b.step)
    gsteps = 20
    g = lbm_sim.Graph(b, gsteps)

    def graph(n):
        assert n % gsteps == 0
        g.launch(n // gsteps)

    ms_graph = timed(graph)
    g.close()
    b.close()
    finite = all(np.isfinite(s.totals()).all() for s in sims)
    for s in sims:
        s.close()

    def rate(ms):
        return round(cells * args.steps / (ms * 1e-3) / 1e6, 1)

    return {
        "metric": "aggregate MLUPS of a batch of independent grids",
        "value": rate(ms_batch),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "dtype": ARITH[args.storage],
        "data": "synthetic",
        "config": {"workload": "%d D2Q37 grids (%s mix, seed %d), %d cells in all, %s storage"
                               % (len(wls), args.mix, args.seed, cells, args.storage.upper()),
                   "grids": [list(wl.dims[:2]) for wl in wls]},
        "sequential_mlups": rate(ms_seq),
        "batched_mlups": rate(ms_batch),
        "batched_graph_mlups": rate(ms_graph),
        "speedup_vs_sequential": round(ms_seq / ms_batch, 3),
        "finite": bool(finite),
    }


def serve_stream(args) -> dict:
    """The serving stream: --count D2Q37 requests, Poisson arrivals at --rate/s,
    --req-steps steps each, served by continuous batching under an HBM budget:
    a latency run in real time, a throughput run with every request queued at
    t = 0, and the same requests solved one after another with the single-grid
    kernel."""
    from paper_2302_04741_amd import serve

    reqs = serve.make_requests(n=args.count, rate=args.rate, seed=args.seed, steps=args.req_steps)
    budget = int(args.budget_gib * (1 << 30))

    def server():
        return serve.Server(storage=args.storage, max_slots=args.slots, budget_bytes=budget,
                            chunk_steps=args.chunk, launch=args.launch)

    live = server().run(reqs, realtime=True)
    print("serve: real-time run done in %.1f s" % live["wall_s"], file=sys.stderr, flush=True)
    thr = server().run(reqs, realtime=False)
    print("serve: queued run done in %.1f s" % thr["wall_s"], file=sys.stderr, flush=True)
    seq = serve.run_sequential(reqs, storage=args.storage)
    print("serve: sequential run done in %.1f s" % seq["wall_s"], file=sys.stderr, flush=True)
    return {
        "workload": "%d D2Q37 requests, Poisson %.0f/s (seed %d), L ~ U{64..1024}, %d steps "
                    "each, %s storage, %d slots, %.1f GiB budget, %d-step chunks"
                    % (args.count, args.rate, args.seed, args.req_steps, args.storage.upper(),
                       args.slots, args.budget_gib, args.chunk),
        "p50_latency_s": round(live["p50_latency_s"], 4),
        "p99_latency_s": round(live["p99_latency_s"], 4),
        "requests": live["requests"],
        "failed": live["failed"],
        "max_concurrent": live["max_concurrent"],
        "live_wall_s": round(live["wall_s"], 3),
        "live_aggregate_mlups": round(live["aggregate_mlups"], 1),
        "queued_aggregate_mlups": round(thr["aggregate_mlups"], 1),
        "queued_wall_s": round(thr["wall_s"], 3),
        "queued_max_concurrent": thr["max_concurrent"],
        "queued_failed": thr["failed"],
        "sequential_aggregate_mlups": round(seq["aggregate_mlups"], 1),
        "sequential_wall_s": round(seq["wall_s"], 3),
        "launch": {"live": live["launches"], "queued": thr["launches"]},
    }


def bench_serve(args) -> dict:
    """The serving stream as its own bench line (p99 latency as the value)."""
    sv = serve_stream(args)
    out = {
        "metric": "served completion latency p50/p99 and aggregate MLUPS",
        "value": sv["p99_latency_s"],
        "unit": "s (p99 latency)",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": ARITH[args.storage],
        "data": "synthetic",
        "config": {"workload": sv.pop("workload")},
    }
    out.update(sv)
    return out


def bench_channel(args) -> dict:
    """The channel of Sec. 3 (D2Q37 3 x 150 between plates, per-cell tau): time
    per step of the plated step kernel, one launch per step, timed with HIP
    events on the handle's stream over --steps steps after --warmup."""
    import torch

    from paper_2302_04741_amd import sim as lbm_sim
    from paper_2302_04741_amd import workloads

    wl = workloads.channel()
    stream = torch.cuda.Stream()
    s = lbm_sim.from_workload(wl, storage=args.storage, stream=stream)
    s.step(args.warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream.synchronize()
    e0.record(stream)
    s.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    s.totals()  # raises on a non-finite state
    s.close()
    return {
        "metric": "channel step time",
        "value": round(us, 3),
        "unit": "us/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": False,
        "dtype": ARITH[args.storage],
        "data": "synthetic",
        "config": {"workload": wl.name + ", per-cell tau, %s storage" % args.storage.upper()},
        "mlups": round(wl.ncell / us, 3),
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid side (default 256)")
    ap.add_argument("--lattice", default="D3Q39", choices=["D3Q39", "D2Q37"],
                    help="step workload: D3Q39 Kolmogorov flow (n^3, the headline) or the "
                         "D2Q37 thermal shear wave (n^2, tau and force of the D2Q37 sweep)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16dev"])
    ap.add_argument("--tau", type=float, default=0.8, help="tau-hat of the step workload")
    ap.add_argument("--block", type=int, default=0, help="threads per block (0 = default)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed regions of --steps steps reported as a spread")
    ap.add_argument("--cpu-steps", type=int, default=6,
                    help="oracle steps of the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter summary under profiles/ and exit (no GPU)")
    ap.add_argument("--workload", default="step", choices=["step", "batch", "serve", "channel"],
                    help="step: the fused step on one grid (default); batch: a mix of "
                         "independent grids, batched vs sequential; serve: the request stream; "
                         "channel: the plated 3 x 150 channel, time per step")
    ap.add_argument("--mix", default="serve", choices=["serve", "small"],
                    help="batch: grid sizes of the serving stream or small grids")
    ap.add_argument("--count", type=int, default=0,
                    help="batch: number of grids (default 64); serve: requests (default 256)")
    ap.add_argument("--seed", type=int, default=4741)
    ap.add_argument("--batch-threads", type=int, default=0,
                    help="batch: threads per block (64, 128, 256; 0 = 128)")
    ap.add_argument("--batch-blocks", type=int, default=0,
                    help="batch: 0 = one block per tile, > 0 = persistent grid")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: arrivals per second")
    ap.add_argument("--req-steps", type=int, default=2000, help="serve: steps per request")
    ap.add_argument("--slots", type=int, default=64, help="serve: concurrent requests")
    ap.add_argument("--budget-gib", type=float, default=1.0, help="serve: HBM budget")
    ap.add_argument("--chunk", type=int, default=25, help="serve: steps per batched chunk")
    ap.add_argument("--launch", default="default", choices=["default", "tuned"],
                    help="serve: multi-grid launch shape (default: 128 threads, one wavefront "
                         "per tile; tuned: the autotuner's choice per batch class)")
    ap.add_argument("--serve-count", type=int, default=256,
                    help="step: requests of the serving stream in the default line")
    ap.add_argument("--no-serve", action="store_true",
                    help="step: leave out the serving-stream figures of the default line")
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

    if args.workload != "step":
        if args.workload == "batch":
            args.count = args.count or 64
            out = bench_batch(args)
        elif args.workload == "channel":
            out = bench_channel(args)
        else:
            args.count = args.count or 256
            out = bench_serve(args)
        print(json.dumps(out), flush=True)
        return 0

    import torch

    from paper_2302_04741_amd import sim as lbm_sim
    from paper_2302_04741_amd import workloads

    if args.lattice == "D3Q39":
        wl = workloads.kolmogorov_3d(n=args.n, tau_hat=args.tau)
    else:
        wl = workloads.thermal_shear_2d(n=args.n, tau_hat=args.tau, dtheta=0.1, mach=0.2)
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
    # further timed regions of the same length, for the spread (median of 5)
    rep_ms = []
    for _ in range(args.repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        rep_ms.append(e0.elapsed_time(e1) / args.steps)
    # the ceiling of the step's access pattern: the same traffic without the
    # arithmetic (lbm_pattern_pass), at each block size, the best one kept (at
    # the step's own shape the bare pattern can be slower than the step: with
    # no arithmetic between them, more loads and stores are in flight at once)
    pat_ms = {}
    if args.repeats > 0:
        for blk in PATTERN_BLOCKS:
            s.set_block(blk)
            best = None
            for _ in range(2):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                s.pattern_pass(args.steps)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                best = ms if best is None else min(best, ms)
            pat_ms[blk] = best
        s.set_block(args.block)
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
    Q = 39 if args.lattice == "D3Q39" else 37
    sbytes = {"f32": 4, "f64": 8, "f16dev": 2}[args.storage]
    ms_per_step = ms_events / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    bytes_per_launch = 2.0 * Q * sbytes * N
    achieved = bytes_per_launch / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic() if (args.lattice == "D3Q39" and args.n == 256
                                     and args.storage == "f32") else None
    if args.lattice == "D3Q39":
        what = ("D3Q39 %d^3 periodic Kolmogorov flow, %s deviation storage, tau=%g, "
                "3rd-order equilibrium, force with a3_F and sigma"
                % (args.n, args.storage.upper(), args.tau))
    else:
        what = ("D2Q37 %d^2 periodic thermal shear wave (dtheta 0.1, Ma 0.2, g = (0, -1e-5)), "
                "%s deviation storage, tau=%g, 4th-order equilibrium, force with a3_F and "
                "sigma" % (args.n, args.storage.upper(), args.tau))

    out = {
        "metric": "%s force-collide-stream MLUPS" % args.lattice,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ARITH[args.storage],
        "data": "synthetic",
        "config": {
            "workload": what,
            "grid": list(wl.dims),
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
    if pat_ms:
        by_block = {str(b): round(bytes_per_launch / (ms * 1e-3) / 1e9, 1)
                    for b, ms in pat_ms.items()}
        pat = max(by_block.values())
        out["pattern_ceiling"] = {
            "achieved": pat, "unit": "GB/s",
            "what": "the step's loads and stores alone, no arithmetic (lbm_pattern_pass), "
                    "best over block sizes, %d passes each" % args.steps,
            "by_block": by_block,
            "step_frac": round(achieved / pat, 4),
        }
    if rep_ms:
        med = sorted(rep_ms)[len(rep_ms) // 2]
        out["repeats"] = {"count": len(rep_ms), "steps_each": args.steps,
                          "median_mlups": round(N / (med * 1e-3) / 1e6, 1),
                          "min_mlups": round(N / (max(rep_ms) * 1e-3) / 1e6, 1),
                          "max_mlups": round(N / (min(rep_ms) * 1e-3) / 1e6, 1)}
    del s, rho, u, th
    torch.cuda.empty_cache()
    if not args.no_serve and args.lattice == "D3Q39":
        # the latency half of the metric: the serving stream (D2Q37 FP32 requests)
        sargs = argparse.Namespace(**vars(args))
        sargs.storage, sargs.count = "f32", args.serve_count
        out["serving"] = serve_stream(sargs)
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
