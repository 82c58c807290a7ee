"""Python handle over the C ABI: torch supplies device memory and streams.

Every step of the method runs in the HIP kernels of liblbm.so; this module only
allocates the workspace and the in/out tensors with torch and passes pointers.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import check, load

DIM = {"D2Q37": 2, "D3Q39": 3}


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required: the library has no CPU path")
    return torch


def _as_device(torch, a, shape, device, stream, keep):
    """float64 contiguous device tensor of `shape` from a tensor or array."""
    if isinstance(a, torch.Tensor) and a.is_cuda:
        t = a.to(device=device, dtype=torch.float64).reshape(shape).contiguous()
    else:
        arr = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))
        t = torch.from_numpy(arr.copy()).to(device=device, non_blocking=False)
    # read on `stream`: keep the memory from being reused before that stream
    # has used it (the caller's tensor itself, or a temporary made here)
    t.record_stream(stream)
    keep.append(t)
    return t


class Sim:
    """One periodic simulation whose populations live in a torch-owned workspace.

    lattice: "D2Q37" or "D3Q39"; dims: (nx, ny[, nz]); tau_hat: relaxation time
    of eq. (lbm); rho, theta: (N,), u: (D, N) initial fields (numpy or torch, any
    device; converted to FP64 on the GPU); cell = (z*ny + y)*nx + x.
    storage: "f64" | "f32" (| "f16dev"); eq_order: 0 = highest supported;
    force_order: 1..4 (4 = full scheme incl. a3_F and sigma); rho0: reference
    density of the stored deviations (default 1; 0 stores f~ itself).
    """

    def __init__(self, lattice: str, dims, tau_hat: float, rho, u, theta, *, storage="f64",
                 eq_order: int = 0, force_order: int = 4, force_field: bool = False,
                 rho0: float | None = None, walls: bool = False, device=None, stream=None):
        torch = _torch()
        L = load()
        self.lattice = lattice
        self.D = DIM[lattice]
        nx, ny, nz = (tuple(int(d) for d in dims) + (1, 1))[:3]
        self.dims = (nx, ny, nz)
        self.N = nx * ny * nz
        self.storage = storage
        if rho0 is None:
            # store deviations from w_i * 1 (rho0 = 0 gives the literal form)
            rho0 = 1.0
        self.rho0 = rho0
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = _lib.make_params(lattice, self.dims, tau_hat, storage, eq_order,
                                       force_order, force_field, rho0, walls)
        nbytes = L.lbm_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            # invalid parameters: let lbm_create report why
            nbytes = 256
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        # the kernels use the workspace on the handle's stream: once freed, the
        # allocator must not hand it out before that stream has finished with it
        raw.record_stream(self.stream)
        self._raw = raw
        self.workspace_bytes = nbytes
        self._ws_ptr = raw.data_ptr() + off
        keep = []
        N, D = self.N, self.D
        self._before()  # inputs made on the caller's stream are ready first
        with torch.cuda.stream(self.stream):
            r = _as_device(torch, rho, (N,), self.device, self.stream, keep)
            uu = _as_device(torch, u, (D, N), self.device, self.stream, keep)
            th = _as_device(torch, theta, (N,), self.device, self.stream, keep)
        handle = ctypes.c_void_p()
        check(L.lbm_create(ctypes.byref(self.params), ctypes.c_void_p(self._ws_ptr),
                           ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                           ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(uu.data_ptr()),
                           ctypes.c_void_p(th.data_ptr()), ctypes.byref(handle)))
        self._h = handle
        del keep  # temporaries are protected by record_stream until the stream has used them

    # -- helpers -------------------------------------------------------------
    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("simulation is closed")
        return self._h

    def _empty(self, *shape):
        torch = _torch()
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    # Stream ordering.  The library runs everything on the handle's stream;
    # tensors handed in or out belong to the caller's current stream.  Before
    # the handle's stream touches such tensors it waits for the current
    # stream; after it wrote them the current stream waits for it, and the
    # allocator is told the tensors were used on the handle's stream.
    def _before(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)
        return cur

    def _after(self, cur, *tensors):
        if cur.cuda_stream != self.stream.cuda_stream:
            for t in tensors:
                t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    # -- the five calls ------------------------------------------------------
    def set_force(self, g=None, *, axis=None, profile=None, field=None):
        """Uniform g (D values), an axis profile (D, L_axis) along `axis`, or a
        full (D, N) field."""
        torch = _torch()
        L = load()
        if g is not None:
            gg = (ctypes.c_double * 3)(*[float(v) for v in np.asarray(g, np.float64).reshape(-1)[:self.D]])
            check(L.lbm_set_force(self.handle, 0, gg, 0, 0))
            return
        keep = []
        self._before()
        with torch.cuda.stream(self.stream):
            self._set_force_device(torch, L, keep, axis, profile, field)

    def _set_force_device(self, torch, L, keep, axis, profile, field):
        if profile is not None:
            prof = np.asarray(profile.cpu() if isinstance(profile, torch.Tensor) else profile,
                              dtype=np.float64).reshape(self.D, -1)
            t = _as_device(torch, prof, prof.shape, self.device, self.stream, keep)
            check(L.lbm_set_force(self.handle, 1, ctypes.c_void_p(t.data_ptr()), int(axis),
                                  prof.shape[1]))
        elif field is not None:
            t = _as_device(torch, field, (self.D, self.N), self.device, self.stream, keep)
            check(L.lbm_set_force(self.handle, 2, ctypes.c_void_p(t.data_ptr()), 0, 0))
        else:
            raise ValueError("give g, profile= (with axis=) or field=")

    def set_workload_force(self, force):
        """Apply a workload force tuple: ("uniform", g) | ("axis", axis, prof) | ("field", g)."""
        kind = force[0]
        if kind == "uniform":
            self.set_force(force[1])
        elif kind == "axis":
            self.set_force(axis=force[1], profile=force[2])
        elif kind == "field":
            self.set_force(field=force[1])
        else:
            raise ValueError(kind)

    def step(self, n: int = 1):
        check(load().lbm_step(self.handle, int(n)))

    def moments(self):
        """(rho (N,), u (D, N), theta (N,)) as float64 device tensors, ready on
        the caller's current stream."""
        rho, u, th = self._empty(self.N), self._empty(self.D, self.N), self._empty(self.N)
        cur = self._before()
        check(load().lbm_moments(self.handle, ctypes.c_void_p(rho.data_ptr()),
                                 ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(th.data_ptr())))
        self._after(cur, rho, u, th)
        return rho, u, th

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lbm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- diagnostics -----------------------------------------------------------
    def heat_flux(self):
        q = self._empty(self.D, self.N)
        cur = self._before()
        check(load().lbm_heat_flux(self.handle, ctypes.c_void_p(q.data_ptr())))
        self._after(cur, q)
        return q

    def totals(self) -> np.ndarray:
        out = (ctypes.c_double * (self.D + 2))()
        check(load().lbm_totals(self.handle, out))
        return np.array(out[:])

    def totals_device(self, out=None):
        """The totals of totals(), as D+2 float64 on the device, enqueued on the
        handle's stream without waiting (no finiteness check); ready on the
        caller's current stream."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.D + 2, dtype=torch.float64, device=self.device)
        cur = self._before()
        check(load().lbm_totals_device(self.handle, ctypes.c_void_p(out.data_ptr())))
        self._after(cur, out)
        return out

    def population_bytes(self) -> int:
        return int(load().lbm_population_bytes(self.handle))

    def get_populations(self):
        torch = _torch()
        t = torch.empty(self.population_bytes(), dtype=torch.uint8, device=self.device)
        cur = self._before()
        check(load().lbm_get_populations(self.handle, ctypes.c_void_p(t.data_ptr())))
        self._after(cur, t)
        return t

    def set_populations(self, t):
        assert t.numel() * t.element_size() == self.population_bytes()
        assert t.is_contiguous() and t.device.type == "cuda"
        cur = self._before()
        check(load().lbm_set_populations(self.handle, ctypes.c_void_p(t.data_ptr())))
        self._after(cur, t)

    @property
    def step_count(self) -> int:
        return int(load().lbm_step_count(self.handle))

    @step_count.setter
    def step_count(self, n: int):
        check(load().lbm_set_step_count(self.handle, int(n)))

    def pattern_pass(self, repeats: int = 1):
        """Diagnostic: `repeats` passes of the step's memory traffic without its
        arithmetic (the state is unchanged); its rate is the ceiling of the
        step's access pattern."""
        check(load().lbm_pattern_pass(self.handle, int(repeats)))

    def set_viscosity(self, mu: float):
        """mu > 0: per-cell relaxation time tau^ = mu/(rho theta) + 1/2 (the
        dynamic viscosity held constant); 0: the constant tau_hat again."""
        check(load().lbm_set_viscosity(self.handle, float(mu)))

    def set_walls(self, theta_b: float, theta_t: float, u_b: float = 0.0, u_t: float = 0.0,
                  enable: bool = True):
        """Plates at y = -1/2 and y = ny - 1/2 with temperatures and tangential
        velocities (needs walls=True at creation and step count 0)."""
        check(load().lbm_set_walls(self.handle, int(bool(enable)), float(theta_b),
                                   float(theta_t), float(u_b), float(u_t)))

    def set_block(self, threads: int):
        check(load().lbm_set_block(self.handle, int(threads)))

    def set_stream(self, stream):
        check(load().lbm_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))
        self._raw.record_stream(stream)
        self.stream = stream


def from_workload(wl, storage="f64", **kw) -> Sim:
    """Create a Sim for a workloads.Workload and apply its force."""
    force_field = wl.force[0] == "field"
    s = Sim(wl.lattice, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta, storage=storage,
            eq_order=wl.eq_order, force_order=wl.force_order, force_field=force_field,
            walls=wl.walls is not None, **kw)
    if wl.mu > 0:
        s.set_viscosity(wl.mu)
    s.set_workload_force(wl.force)
    if wl.walls is not None:
        # last: the state is rebuilt from the moments, which equal the inputs
        # only while the grid is periodic
        s.set_walls(*wl.walls)
    return s


class Graph:
    """A captured loop of `nsteps` (even) steps of a Sim or a Batch (HIP graph)."""

    def __init__(self, target, nsteps: int):
        L = load()
        h = ctypes.c_void_p()
        if isinstance(target, Sim):
            check(L.lbm_graph_create(target.handle, None, int(nsteps), ctypes.byref(h)))
        else:
            check(L.lbm_graph_create(None, target.handle, int(nsteps), ctypes.byref(h)))
        self._h = h
        self.nsteps = int(nsteps)
        self.target = target

    def launch(self, repeats: int = 1):
        if isinstance(self.target, Batch):
            self.target._pre()
        check(load().lbm_graph_launch(self._h, int(repeats)))
        if isinstance(self.target, Batch):
            self.target._post()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lbm_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several Sims advanced together by the multi-grid kernel: one launch per
    step for all members (same lattice, storage and orders; any grid sizes,
    relaxation times, forces and plates)."""

    def __init__(self, max_sims: int, device=None, stream=None):
        torch = _torch()
        L = load()
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.lbm_batch_workspace_bytes(int(max_sims))
        if nbytes == 0:
            raise ValueError("max_sims out of range")
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        raw.record_stream(self.stream)
        self._raw = raw
        ws = raw.data_ptr() + (-raw.data_ptr()) % 256
        h = ctypes.c_void_p()
        check(L.lbm_batch_create(int(max_sims), ctypes.c_void_p(ws), ctypes.c_size_t(nbytes),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.members = []
        self._member_streams = {}

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("batch is closed")
        return self._h

    def _pre(self):
        for st in self._member_streams.values():
            self.stream.wait_stream(st)

    def _post(self):
        for st in self._member_streams.values():
            st.wait_stream(self.stream)

    def set(self, sims):
        arr = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
        check(load().lbm_batch_set(self.handle, arr, len(sims)))
        self.members = list(sims)
        self._member_streams = {}
        for s in sims:
            if s.stream.cuda_stream != self.stream.cuda_stream:
                self._member_streams[s.stream.cuda_stream] = s.stream

    def step(self, n: int = 1):
        # members may run their own work on other streams: order the batch's
        # launches after it, and their later work after the batch
        self._pre()
        check(load().lbm_batch_step(self.handle, int(n)))
        self._post()

    def set_launch(self, threads: int = 0, blocks: int = 0):
        """Threads per block (64, 128, 256; 0 = 128) and grid (0 = one
        wavefront per 64-cell tile, > 0 = persistent grid of that many blocks)."""
        check(load().lbm_batch_set_launch(self.handle, int(threads), int(blocks)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lbm_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step_noalloc(sims, n: int = 1, stream=None):
    """Advance `sims` (1..256 Sims sharing lattice, storage and orders) by n
    steps of the multi-grid kernel without a batch handle or workspace: the
    tile table lives in the library's fixed device array
    (lbm_batch_step_noalloc; calls that overlap on one device race).  Runs on
    `stream` (default: the current stream), ordered after the members' own
    streams and before their later work."""
    torch = _torch()
    if not sims:
        raise ValueError("no simulations")
    stream = stream if stream is not None else torch.cuda.current_stream(sims[0].device)
    others = {s.stream.cuda_stream: s.stream for s in sims
              if s.stream.cuda_stream != stream.cuda_stream}
    for st in others.values():
        stream.wait_stream(st)
    arr = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
    check(load().lbm_batch_step_noalloc(arr, len(sims), int(n),
                                        ctypes.c_void_p(stream.cuda_stream)))
    for st in others.values():
        st.wait_stream(stream)


def round_f16_stochastic(v, seed, stream=None):
    """The F16 storage's stochastic rounding (lbm_round_f16_stochastic) of a
    float32 CUDA tensor `v` with the uint32 random words `seed` (an int32 or
    uint32 CUDA tensor of the same size); returns the binary16 results as a
    float16 tensor of v's shape, enqueued on `stream` (default: the current
    stream)."""
    torch = _torch()
    if v.dtype != torch.float32 or not v.is_cuda:
        raise TypeError("v must be a float32 CUDA tensor")
    if seed.dtype not in (torch.int32, torch.uint32) or seed.device != v.device:
        raise TypeError("seed must be an int32/uint32 tensor on v's device")
    if seed.numel() != v.numel():
        raise ValueError("seed and v differ in size")
    v, seed = v.contiguous(), seed.contiguous()
    out = torch.empty(v.shape, dtype=torch.float16, device=v.device)
    stream = stream if stream is not None else torch.cuda.current_stream(v.device)
    check(load().lbm_round_f16_stochastic(ctypes.c_void_p(v.data_ptr()),
                                          ctypes.c_void_p(seed.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), int(v.numel()),
                                          ctypes.c_void_p(stream.cuda_stream)))
    return out
