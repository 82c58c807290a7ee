"""Continuous-batching server of independent simulations.

Requests (a grid, a relaxation time, a force, initial fields and a number of
steps) arrive over time.  The server admits a request as soon as a slot and
enough of its HBM budget are free, keeps every admitted simulation's
populations resident in its own workspace, and advances all admitted
simulations together: each chunk of steps is one launch per step of the
persistent multi-grid kernel over every member (the batch is re-formed
whenever membership changes).  Requests that arrive while others run join at
the next chunk boundary; finished requests release their slot and memory at
once.  A member that diverges (non-finite totals) fails alone and is evicted.

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
    def __init__(self, storage: str = "f32", max_slots: int = 64,
                 budget_bytes: int = 16 << 30, chunk_steps: int = 100,
                 keep_populations: Callable[[int], bool] = lambda rid: False,
                 batch_threads: int = 0, batch_blocks: int = 0, check_every: int = 5):
        self.storage = storage
        self.check_every = max(1, int(check_every))
        self.adm = Admission(max_slots, budget_bytes)
        self.chunk = int(chunk_steps)
        self.keep = keep_populations
        self.batch_threads = batch_threads
        self.batch_blocks = batch_blocks

    def run(self, requests: List[Request], realtime: bool = True) -> Dict[str, object]:
        """Serve `requests`.  realtime=True honours the arrival times (latency
        run); realtime=False makes every request available at t = 0
        (throughput run)."""
        import torch

        from . import sim

        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            if request_bytes(r, self.storage) > self.adm.budget:
                raise ValueError("request %d needs more than the whole budget" % r.rid)
        active = []   # dicts: req, sim, bytes, admitted, done
        results: List[Result] = []
        batch = sim.Batch(self.adm.max_slots)
        if self.batch_threads or self.batch_blocks:
            batch.set_launch(self.batch_threads, self.batch_blocks)
        members = None
        t0 = time.perf_counter()
        lu = 0
        max_active = 0
        chunks = 0

        def now():
            return time.perf_counter() - t0

        while pending or active:
            t = now()
            # admit in arrival order while a slot and the budget allow
            while pending and (not realtime or pending[0].arrival <= t):
                r = pending[0]
                nb = request_bytes(r, self.storage)
                if not self.adm.fits(nb):
                    break
                pending.pop(0)
                self.adm.take(nb)
                s = sim.from_workload(r.workload, storage=self.storage)
                active.append({"req": r, "sim": s, "bytes": nb,
                               "admitted": now() if realtime else 0.0, "done": 0})
            max_active = max(max_active, len(active))
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.01)))
                continue
            ids = [a["req"].rid for a in active]  # unique per admission
            if ids != members:
                batch.set([a["sim"] for a in active])
                members = ids
            n = min(self.chunk, min(a["req"].steps - a["done"] for a in active))
            batch.step(n)
            for a in active:
                a["done"] += n
                lu += a["req"].workload.ncell * n
            torch.cuda.current_stream().synchronize()
            chunks += 1
            check_all = chunks % self.check_every == 0
            still = []
            for a in active:
                r = a["req"]
                finished = a["done"] >= r.steps
                err = ""
                totals = None
                if finished or check_all:
                    try:
                        totals = a["sim"].totals()  # raises on a non-finite state
                    except Exception as e:  # a diverged member fails alone
                        err = str(e)
                if finished or err:
                    pops = a["sim"].get_populations().cpu() if (self.keep(r.rid) and not err) \
                        else None
                    results.append(Result(r.rid, r.arrival if realtime else 0.0, a["admitted"],
                                          now(), r.workload.ncell, a["done"], not err, err,
                                          totals, pops))
                    a["sim"].close()
                    self.adm.release(a["bytes"])
                else:
                    still.append(a)
            active = still
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
