"""ctypes binding of liblbm.so (the C ABI declared in include/lbm.h).

Argument marshalling only.  The library must be built (``build.build()``);
nothing here falls back to another implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
LBM_EINVAL = -1
LBM_EUNSUPPORTED = -2
LBM_EDEVICE = -3
LBM_ENOSPACE = -4
LBM_ENONFINITE = -5
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_EUNSUPPORTED", -3: "LBM_EDEVICE",
                -4: "LBM_ENOSPACE", -5: "LBM_ENONFINITE"}

LATTICES = {"D2Q37": 0, "D3Q39": 1}
STORAGES = {"f64": 0, "f32": 1, "f16dev": 2}
FORCE_KINDS = {"uniform": 0, "axis": 1, "field": 2}
FLAG_FORCE_FIELD = 1
FLAG_WALLS = 2
NOALLOC_MAX_SIMS = 256  # LBM_NOALLOC_MAX_SIMS

#: the C-ABI entry points, in the order include/lbm.h declares them
API_SYMBOLS = (
    "lbm_workspace_bytes", "lbm_create", "lbm_set_force", "lbm_step", "lbm_moments",
    "lbm_destroy", "lbm_last_error", "lbm_totals", "lbm_totals_device", "lbm_heat_flux", "lbm_pattern_pass",
    "lbm_round_f16_stochastic",
    "lbm_population_bytes",
    "lbm_get_populations", "lbm_set_populations", "lbm_step_count", "lbm_set_step_count",
    "lbm_set_stream", "lbm_set_block", "lbm_set_viscosity",
    "lbm_set_walls", "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_set",
    "lbm_batch_step", "lbm_batch_set_launch", "lbm_batch_destroy", "lbm_batch_step_noalloc",
    "lbm_graph_create", "lbm_graph_launch", "lbm_graph_destroy", "lbm_lattice_table",
    "lbm_version",
)


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("lattice", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("eq_order", ctypes.c_int32),
        ("force_order", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("tau_hat", ctypes.c_double),
        ("rho0", ctypes.c_double),
    ]


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, message))


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)


def load() -> ctypes.CDLL:
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblbm.so is not built (run paper_2302_04741_amd.build.build()); "
                          "there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    pp = ctypes.POINTER(lbm_params)
    L.lbm_workspace_bytes.argtypes = [pp]
    L.lbm_workspace_bytes.restype = _sz
    L.lbm_create.argtypes = [pp, _vp, _sz, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]
    L.lbm_create.restype = _i32
    L.lbm_set_force.argtypes = [_vp, _i32, _vp, _i32, _i64]
    L.lbm_set_force.restype = _i32
    L.lbm_step.argtypes = [_vp, _i64]
    L.lbm_step.restype = _i32
    L.lbm_moments.argtypes = [_vp, _vp, _vp, _vp]
    L.lbm_moments.restype = _i32
    L.lbm_destroy.argtypes = [_vp]
    L.lbm_destroy.restype = None
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_totals.argtypes = [_vp, _dp]
    L.lbm_totals.restype = _i32
    L.lbm_totals_device.argtypes = [_vp, _vp]
    L.lbm_totals_device.restype = _i32
    L.lbm_heat_flux.argtypes = [_vp, _vp]
    L.lbm_round_f16_stochastic.argtypes = [_vp, _vp, _vp, _i64, _vp]
    L.lbm_round_f16_stochastic.restype = _i32
    L.lbm_heat_flux.restype = _i32
    L.lbm_pattern_pass.argtypes = [_vp, _i64]
    L.lbm_pattern_pass.restype = _i32
    L.lbm_population_bytes.argtypes = [_vp]
    L.lbm_population_bytes.restype = _sz
    L.lbm_get_populations.argtypes = [_vp, _vp]
    L.lbm_get_populations.restype = _i32
    L.lbm_set_populations.argtypes = [_vp, _vp]
    L.lbm_set_populations.restype = _i32
    L.lbm_step_count.argtypes = [_vp]
    L.lbm_step_count.restype = _i64
    L.lbm_set_step_count.argtypes = [_vp, _i64]
    L.lbm_set_step_count.restype = _i32
    L.lbm_set_stream.argtypes = [_vp, _vp]
    L.lbm_set_stream.restype = _i32
    L.lbm_set_block.argtypes = [_vp, _i32]
    L.lbm_set_block.restype = _i32
    L.lbm_set_viscosity.argtypes = [_vp, ctypes.c_double]
    L.lbm_set_viscosity.restype = _i32
    _d = ctypes.c_double
    L.lbm_set_walls.argtypes = [_vp, _i32, _d, _d, _d, _d]
    L.lbm_set_walls.restype = _i32
    L.lbm_batch_workspace_bytes.argtypes = [_i32]
    L.lbm_batch_workspace_bytes.restype = _sz
    L.lbm_batch_create.argtypes = [_i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]
    L.lbm_batch_create.restype = _i32
    L.lbm_batch_set.argtypes = [_vp, ctypes.POINTER(_vp), _i32]
    L.lbm_batch_set.restype = _i32
    L.lbm_batch_step.argtypes = [_vp, _i64]
    L.lbm_batch_step.restype = _i32
    L.lbm_batch_set_launch.argtypes = [_vp, _i32, _i64]
    L.lbm_batch_set_launch.restype = _i32
    L.lbm_batch_destroy.argtypes = [_vp]
    L.lbm_batch_destroy.restype = None
    L.lbm_batch_step_noalloc.argtypes = [ctypes.POINTER(_vp), _i32, _i64, _vp]
    L.lbm_batch_step_noalloc.restype = _i32
    L.lbm_graph_create.argtypes = [_vp, _vp, _i64, ctypes.POINTER(_vp)]
    L.lbm_graph_create.restype = _i32
    L.lbm_graph_launch.argtypes = [_vp, _i64]
    L.lbm_graph_launch.restype = _i32
    L.lbm_graph_destroy.argtypes = [_vp]
    L.lbm_graph_destroy.restype = None
    L.lbm_lattice_table.argtypes = [_i32, ctypes.POINTER(_i32), _dp, _dp]
    L.lbm_lattice_table.restype = _i32
    L.lbm_version.argtypes = []
    L.lbm_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int) -> int:
    if status < 0:
        raise LbmError(status, load().lbm_last_error().decode())
    return status


def make_params(lattice: str, dims, tau_hat: float, storage: str = "f64", eq_order: int = 0,
                force_order: int = 4, force_field: bool = False, rho0: float = 1.0,
                walls: bool = False) -> lbm_params:
    nx, ny, nz = (tuple(int(d) for d in dims) + (1, 1))[:3]
    p = lbm_params()
    p.struct_size = ctypes.sizeof(lbm_params)
    p.lattice = LATTICES[lattice] if isinstance(lattice, str) else int(lattice)
    p.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
    p.eq_order = int(eq_order)
    p.force_order = int(force_order)
    p.flags = (FLAG_FORCE_FIELD if force_field else 0) | (FLAG_WALLS if walls else 0)
    p.nx, p.ny, p.nz = nx, ny, nz
    p.tau_hat = float(tau_hat)
    p.rho0 = float(rho0)
    return p


def workspace_bytes(p: lbm_params) -> int:
    return int(load().lbm_workspace_bytes(ctypes.byref(p)))


def lattice_table(lattice: str):
    """(c (Q,3) ints, w (Q,), r) of the velocity set compiled into the library."""
    import numpy as np

    L = load()
    lat = LATTICES[lattice]
    c = (ctypes.c_int32 * (64 * 3))()
    w = (ctypes.c_double * 64)()
    r = ctypes.c_double()
    Q = check(L.lbm_lattice_table(lat, c, w, ctypes.byref(r)))
    cc = np.frombuffer(c, dtype=np.int32, count=3 * Q).reshape(Q, 3).copy()
    ww = np.frombuffer(w, dtype=np.float64, count=Q).copy()
    return cc, ww, r.value
