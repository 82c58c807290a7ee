"""Autotuner of launch shapes.

* Single-grid step: threads per block (64 ... 1024) per (lattice, storage,
  equilibrium order, force order, grid class).
* Multi-grid (batched) step: threads per block and grid (one wavefront per
  tile or a persistent grid) per (lattice, storage, orders, batch class).

Candidates are timed with HIP events on scratch simulations of the same shape
(smooth synthetic fields; the cost of a step does not depend on the data), so
tuning never touches a caller's state.  Results are cached in a JSON file
(``$LBM_AUTOTUNE_CACHE``, default ``~/.cache/paper_2302_04741_amd/autotune.json``),
keyed by the GPU architecture and the library version as well as the problem class.
Every launch shape gives bitwise the same results, so tuning only affects speed.
"""
from __future__ import annotations

import json
import os
import threading

BLOCK_CANDIDATES = (64, 128, 256, 512, 1024)
# (threads per block, blocks: 0 = one wavefront per tile, else a persistent grid)
BATCH_CANDIDATES = ((64, 0), (128, 0), (256, 0), (256, 1280), (256, 2560), (64, 5120))

_lock = threading.Lock()


def cache_path() -> str:
    return os.path.expanduser(os.environ.get(
        "LBM_AUTOTUNE_CACHE", "~/.cache/paper_2302_04741_amd/autotune.json"))


def _bucket(n: int) -> int:
    b = 1
    while b < n:
        b *= 2
    return b


def grid_class(dims) -> str:
    nx, ny, nz = (tuple(int(d) for d in dims) + (1, 1))[:3]
    return "x%d_r%d" % (_bucket(nx), _bucket(ny * nz))


def batch_class(dims_list) -> str:
    cells = sum(int(d[0]) * int(d[1]) * (int(d[2]) if len(d) > 2 else 1) for d in dims_list)
    return "n%d_c%d" % (_bucket(len(dims_list)), _bucket(cells))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, value) -> None:
    with _lock:
        data = _load_cache()
        data[key] = value
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)


def _time_steps(torch, step, stream, steps: int) -> float:
    step(2)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _scratch(lattice, dims, storage, eq_order, force_order, seed=0, stream=None):
    from . import sim, workloads

    wl = workloads.random_smooth(lattice, tuple(dims), seed=seed, force_kind="uniform",
                                 force_order=force_order)
    wl.eq_order = eq_order
    return sim.from_workload(wl, storage=storage, stream=stream)


def _device_tag() -> str:
    """The GPU architecture and the library version: tuned shapes are kept per
    device type and per build of the kernels."""
    import torch

    from . import _lib

    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or props.name
    return "%s/%s" % (arch.split(":")[0], _lib.load().lbm_version().decode())


def block_key(lattice, storage, eq_order, force_order, dims) -> str:
    return "block/%s/%s/%s/eq%d/fo%d/%s" % (_device_tag(), lattice, storage, eq_order,
                                            force_order, grid_class(dims))


def tune_block(lattice: str, dims, storage: str = "f32", eq_order: int = 0, force_order: int = 4,
               steps: int = 10, retune: bool = False) -> int:
    """Fastest threads-per-block for this class of grid (cached)."""
    key = block_key(lattice, storage, eq_order, force_order, dims)
    if not retune:
        hit = _load_cache().get(key)
        if hit:
            return int(hit["block"])
    import torch

    s = _scratch(lattice, dims, storage, eq_order, force_order)
    times = {}
    for b in BLOCK_CANDIDATES:
        if storage == "f64" and b > 256:
            continue  # FP64 blocks are capped at 256 threads
        s.set_block(b)
        times[b] = _time_steps(torch, s.step, s.stream, steps)
    s.close()
    best = min(times, key=times.get)
    _store(key, {"block": best, "ms_per_step": times})
    return best


def batch_key(lattice, storage, eq_order, force_order, dims_list) -> str:
    return "batch/%s/%s/%s/eq%d/fo%d/%s" % (_device_tag(), lattice, storage, eq_order,
                                            force_order, batch_class(dims_list))


def tune_batch_launch(lattice: str, dims_list, storage: str = "f32", eq_order: int = 0,
                      force_order: int = 4, steps: int = 10, retune: bool = False):
    """Fastest (threads, blocks) launch of the multi-grid kernel for this class
    of batch (cached)."""
    key = batch_key(lattice, storage, eq_order, force_order, dims_list)
    if not retune:
        hit = _load_cache().get(key)
        if hit:
            return tuple(hit["launch"])
    import torch

    from . import sim

    stream = torch.cuda.Stream()
    sims = [_scratch(lattice, d, storage, eq_order, force_order, seed=k, stream=stream)
            for k, d in enumerate(dims_list)]
    b = sim.Batch(len(sims), stream=stream)
    b.set(sims)
    times = {}
    for threads, blocks in BATCH_CANDIDATES:
        b.set_launch(threads, blocks)
        times["%d/%d" % (threads, blocks)] = _time_steps(torch, b.step, stream, steps)
    b.close()
    for s in sims:
        s.close()
    best = min(times, key=times.get)
    launch = tuple(int(v) for v in best.split("/"))
    _store(key, {"launch": list(launch), "ms_per_step": times})
    return launch
