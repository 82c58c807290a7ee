"""Continuous-batching server of independent simulations.

Requests (a grid, a relaxation time, a force, initial fields and a number of
steps) arrive over time.  The server admits a request as soon as a slot and
enough of its HBM budget are free, keeps every admitted simulation's
populations resident in its own workspace, and advances all admitted
simulations together: each chunk of steps is one launch per step of the
multi-grid kernel over every member (the batch is re-formed whenever
membership changes).  Requests that arrive while others run join at the next
chunk boundary; finished requests release their slot and memory as soon as
their last chunk has run.  A member that diverges (non-finite totals) fails
alone and is evicted.  Host and device are pipelined: the next chunk is queued
before the host waits for the previous one.

All members of one server share lattice, storage and orders (the multi-grid
kernel is compiled per combination); grid sizes, tau_hat and forces differ.
A member's result does not depend on the other members: the kernel reduces
nothing across cells, so a request gives bitwise the same populations alone
and in any mix.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import workloads

SERVE_SEED = 4741


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    workload: workloads.Workload
    steps: int


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    cells: int
    steps: int
    ok: bool
    error: str = ""
    totals: Optional[np.ndarray] = None
    populations: Optional[object] = None  # torch uint8 tensor when kept
    admitted_chunk: int = 0  # chunks the server had queued before admitting it

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_requests(n: int = 256, rate: float = 20.0, seed: int = SERVE_SEED, steps: int = 2000,
                  lmin: int = 64, lmax: int = 1024) -> List[Request]:
    """The serving workload: Poisson arrivals at `rate` per second; per request a
    square D2Q37 grid of side L ~ U{lmin..lmax}, |g| log-uniform in
    [1e-6, 1e-4] with a uniformly random direction, Ma ~ U[0.05, 0.3],
    dtheta ~ U[0.01, 0.1], tau_hat ~ U[0.55, 1.0], and the thermal-shear
    initial fields (theta = 1 + dtheta sin, u_x = Ma sqrt(theta) sin)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += float(rng.exponential(1.0 / rate))
        L = int(rng.integers(lmin, lmax + 1))
        gmag = 10.0 ** float(rng.uniform(-6.0, -4.0))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        g = (gmag * math.cos(ang), gmag * math.sin(ang))
        mach = float(rng.uniform(0.05, 0.3))
        dth = float(rng.uniform(0.01, 0.1))
        tau = float(rng.uniform(0.55, 1.0))
        wl = workloads.thermal_shear_2d(n=L, tau_hat=tau, dtheta=dth, mach=mach, g=g,
                                        steps=steps)
        out.append(Request(rid, t, wl, steps))
    return out


class Admission:
    """Slot and HBM-budget accounting (host only)."""

    def __init__(self, max_slots: int, budget_bytes: int):
        self.max_slots = int(max_slots)
        self.budget = int(budget_bytes)
        self.used = 0
        self.slots = 0

    def fits(self, nbytes: int) -> bool:
        return self.slots < self.max_slots and self.used + nbytes <= self.budget

    def take(self, nbytes: int) -> None:
        assert self.fits(nbytes)
        self.used += nbytes
        self.slots += 1

    def release(self, nbytes: int) -> None:
        self.used -= nbytes
        self.slots -= 1
        assert self.used >= 0 and self.slots >= 0


def request_bytes(req: Request, storage: str) -> int:
    """HBM a request holds while admitted: its workspace."""
    from . import _lib

    wl = req.workload
    # the same flags sim.from_workload creates the handle with
    p = _lib.make_params(wl.lattice, wl.dims, wl.tau_hat, storage, wl.eq_order, wl.force_order,
                         force_field=wl.force[0] == "field", walls=wl.walls is not None)
    return _lib.workspace_bytes(p) + 256


class Server:
    """Continuous batching on one dedicated stream, pipelined with the host.

    Each loop iteration admits the requests that have arrived (their handles are
    built on a side stream, so the host copies never wait for queued steps),
    re-forms the batch if membership changed (the tile table is written by
    kernels on the serving stream, no host wait), enqueues one chunk of steps
    and, behind it, the FP64 conservation totals of the members that finish or
    are due for a check, copied to pinned host memory.  The host then waits
    only for the chunk before the one just queued, so the device always has the
    next chunk to run while the host retires finished requests (totals checked,
    slot and memory released) and admits new ones.

    launch: "default" (128 threads, one wavefront per 64-cell tile), "tuned"
    (the autotuner's choice for the batch class, tuned on first use and cached),
    or a (threads, blocks) pair applied to every batch.  check_every: chunks
    between the conservation checks of running members (finishing members are
    always checked).  inflight: chunks queued on the device before the host
    waits for the oldest.
    """

    def __init__(self, storage: str = "f32", max_slots: int = 64,
                 budget_bytes: int = 16 << 30, chunk_steps: int = 25,
                 keep_populations: Callable[[int], bool] = lambda rid: False,
                 launch="default", check_every: int = 20, inflight: int = 3):
        self.storage = storage
        self.check_every = max(1, int(check_every))
        self.adm = Admission(max_slots, budget_bytes)
        self.chunk = int(chunk_steps)
        self.keep = keep_populations
        self.launch = launch
        self.inflight = max(1, int(inflight))
        self.launches_used: Dict[str, int] = {}

    def _launch_for(self, sims):
        if self.launch == "default":
            return (0, 0)
        if self.launch == "tuned":
            from . import autotune

            s0 = sims[0]
            return tuple(autotune.tune_batch_launch(
                s0.lattice, [s.dims for s in sims], storage=self.storage,
                eq_order=int(s0.params.eq_order), force_order=int(s0.params.force_order)))
        return tuple(self.launch)

    def run(self, requests: List[Request], realtime: bool = True) -> Dict[str, object]:
        """Serve `requests`.  realtime=True honours the arrival times (latency
        run); realtime=False makes every request available at t = 0
        (throughput run)."""
        import collections

        import torch

        from . import sim

        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            if request_bytes(r, self.storage) > self.adm.budget:
                raise ValueError("request %d needs more than the whole budget" % r.rid)
        self.launches_used = {}
        stream = torch.cuda.Stream()   # every step, table and totals launch of the loop
        side = torch.cuda.Stream()     # building admitted handles
        batch = sim.Batch(self.adm.max_slots, stream=stream)
        width = 5  # D + 2 totals per member, D <= 3
        # one totals buffer per chunk that can be outstanding, plus the one being filled
        ring = [(torch.empty((self.adm.max_slots, width), dtype=torch.float64, device="cuda"),
                 torch.empty((self.adm.max_slots, width), dtype=torch.float64, pin_memory=True))
                for _ in range(self.inflight + 1)]
        active = []   # dicts: req, sim, bytes, admitted, planned (steps enqueued)
        inflight = collections.deque()  # (event, members ending, [(member, row)], ring slot)
        results: List[Result] = []
        members = None
        cur_launch = (0, 0)
        t0 = time.perf_counter()
        lu = 0
        max_active = 0
        chunks = 0
        slot = 0

        def now():
            return time.perf_counter() - t0

        def finish(a, err=""):
            r = a["req"]
            pops = None
            if self.keep(r.rid) and not err:
                with torch.cuda.stream(stream):
                    pops = a["sim"].get_populations().cpu()
            results.append(Result(r.rid, r.arrival if realtime else 0.0, a["admitted"], now(),
                                  r.workload.ncell, a["planned"], not err, err,
                                  a.get("totals"), pops, a["admitted_chunk"]))
            # the workspace is recorded on the serving stream: its memory is not
            # reused before the chunks already queued with it have run
            a["sim"].close()
            self.adm.release(a["bytes"])
            active.remove(a)

        def retire():
            """Wait for the oldest outstanding chunk; check its totals, release
            the requests it finished and those whose state is not finite."""
            ev, ending, checks, k = inflight.popleft()
            ev.synchronize()
            host = ring[k][1]
            for a, row in checks:
                tot = host[row, :a["sim"].D + 2].numpy().copy()
                a["totals"] = tot
                if not np.all(np.isfinite(tot)) and a in active:
                    # a diverged member fails alone (the chunk queued after
                    # this one may still carry it; its result is discarded)
                    finish(a, "non-finite totals at step %d" % a["checked_at"])
            for a in ending:
                if a in active:
                    finish(a)

        while pending or active or inflight:
            t = now()
            # admit in arrival order while a slot and the budget allow; handles
            # are built on the side stream, so the host copies of the initial
            # fields never wait for queued chunks
            while pending and (not realtime or pending[0].arrival <= t):
                r = pending[0]
                nb = request_bytes(r, self.storage)
                if not self.adm.fits(nb):
                    break
                pending.pop(0)
                self.adm.take(nb)
                with torch.cuda.stream(side):
                    s = sim.from_workload(r.workload, storage=self.storage, stream=side)
                stream.wait_stream(side)
                s.set_stream(stream)
                a = {"req": r, "sim": s, "bytes": nb, "admitted": now() if realtime else 0.0,
                     "planned": 0, "admitted_chunk": chunks}
                active.append(a)
                if r.steps <= 0:
                    finish(a)
            max_active = max(max_active, len(active))
            runnable = [a for a in active if a["planned"] < a["req"].steps]
            if runnable:
                with torch.cuda.stream(stream):
                    ids = [a["req"].rid for a in runnable]
                    if ids != members:
                        sims = [a["sim"] for a in runnable]
                        want = self._launch_for(sims)
                        if want != cur_launch:
                            batch.set_launch(*want)
                            cur_launch = want
                        batch.set(sims)
                        members = ids
                    key = "%d threads, %s" % (cur_launch[0] or 128,
                                              "one wavefront per tile" if cur_launch[1] == 0
                                              else "persistent, %d blocks" % cur_launch[1])
                    self.launches_used[key] = self.launches_used.get(key, 0) + 1
                    n = min(self.chunk, min(a["req"].steps - a["planned"] for a in runnable))
                    batch.step(n)
                    chunks += 1
                    check_all = chunks % self.check_every == 0
                    ending, checks = [], []
                    dev, host = ring[slot]
                    for a in runnable:
                        a["planned"] += n
                        lu += a["req"].workload.ncell * n
                        done = a["planned"] >= a["req"].steps
                        if done:
                            ending.append(a)
                        if done or check_all:
                            a["sim"].totals_device(out=dev[len(checks), :a["sim"].D + 2])
                            a["checked_at"] = a["planned"]
                            checks.append((a, len(checks)))
                    if checks:
                        host[:len(checks)].copy_(dev[:len(checks)], non_blocking=True)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                inflight.append((ev, ending, checks, slot))
                slot = (slot + 1) % len(ring)
                # keep the newest inflight - 1 chunks queued behind the one the
                # device runs; retire the older ones
                while len(inflight) > self.inflight - 1:
                    retire()
                continue
            if inflight:
                retire()
                continue
            if pending and realtime:
                time.sleep(max(0.0, min(pending[0].arrival - now(), 0.005)))
        wall = now()
        batch.close()
        lat = np.array([r.latency for r in results if r.ok])
        out = {
            "requests": len(results),
            "failed": int(sum(not r.ok for r in results)),
            "wall_s": wall,
            "lattice_updates": lu,
            "aggregate_mlups": lu / wall / 1e6,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "max_concurrent": max_active,
            "chunks": chunks,
            "launches": dict(self.launches_used),
            "results": results,
        }
        return out


def run_sequential(requests: List[Request], storage: str = "f32") -> Dict[str, object]:
    """Baseline: every request solved alone with the plain single-grid kernel,
    one after another, all available at t = 0."""
    import torch

    from . import sim

    t0 = time.perf_counter()
    lu = 0
    for r in requests:
        s = sim.from_workload(r.workload, storage=storage)
        s.step(r.steps)
        torch.cuda.current_stream().synchronize()
        lu += r.workload.ncell * r.steps
        s.close()
    wall = time.perf_counter() - t0
    return {"requests": len(requests), "wall_s": wall, "lattice_updates": lu,
            "aggregate_mlups": lu / wall / 1e6}
