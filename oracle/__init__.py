"""FP64 CPU oracle of the thermal LBM step with Hermite body force (ctypes shim).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (the HIP path) never imports, links or calls it, and this package never
imports the product package.  The C source derives its own quadrature rule and
Hermite tensors; see the header of ``lbm_oracle.c`` for what each function
follows in the paper (Li & Shan, arXiv:2302.04741, Sec. 2: eqs. (fN), (F),
(f3), (fi), (lbm) and the mid-point stress).

Layouts used here (the oracle's own; they need not match the GPU library):
  * fields are SoA numpy arrays: rho (N,), u (D, N), theta (N,), g (D, N);
  * populations are AoS: f (N, Q), cell = (z*ny + y)*nx + x;
  * the body force is always a full (D, N) field; ``g_uniform`` and
    ``g_axis_profile`` expand the two other force kinds into one.

Precision: ``prec="f64"`` (the oracle proper, binary64) or ``prec="ld"``, the
same source built with x87 80-bit long double.  The 80-bit build exists only to
measure how far the binary64 oracle itself drifts from a more precise run of
the same algorithm (its rounding floor); parity claims are against "f64".

Force orders: 1 = first Hermite term only, 2 = up to the second (the
Guo-equivalent scheme, "without a3_F"), 3 = up to the third without the stress
term, 4 = up to the third including sigma-bar (the full scheme).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIBS = {"f64": os.path.join(_HERE, "liboracle.so"),
         "ld": os.path.join(_HERE, "liboracle_ld.so")}
_DTYPE = {"f64": np.float64, "ld": np.longdouble}
_CREAL = {"f64": ctypes.c_double, "ld": ctypes.c_longdouble}

D2Q37 = 0
D3Q39 = 1
DIM = {D2Q37: 2, D3Q39: 3}

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_int = ctypes.c_int
_ptr = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math): the
    binary64 build and the 80-bit build of the same source."""
    for prec, path in _LIBS.items():
        if force or not os.path.exists(path):
            tmp = path + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                   "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
            if prec == "ld":
                cmd.insert(1, "-DOR_REAL=long double")
            subprocess.run(cmd, check=True)
            os.replace(tmp, path)
    return _LIBS["f64"]


_libs = {}


def lib(prec: str = "f64"):
    if prec not in _libs:
        path = _LIBS[prec]
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        R = _CREAL[prec]
        L.oracle_lattice.argtypes = [_int, _ptr, _ptr, _ptr, _ptr]
        L.oracle_hermite.argtypes = [_int, _int, _ptr]
        L.oracle_maxwell_coeff.argtypes = [_int, _int, R, _ptr, R, _ptr]
        L.oracle_equilibrium.argtypes = [_int, _int, R, _ptr, R, _ptr]
        L.oracle_force.argtypes = [_int, _int, R, _ptr, R, _ptr, _ptr, _ptr]
        L.oracle_init.argtypes = [_int, _i64, _i64, _i64, _int, _int, _ptr,
                                  _ptr, _ptr, _ptr, _ptr, _ptr, _int]
        L.oracle_step.argtypes = [_int, _i64, _i64, _i64, R, R, _int, _int, _ptr,
                                  _ptr, _ptr, _ptr, _i64, _int]
        L.oracle_moments.argtypes = [_int, _i64, _ptr, _ptr, _ptr, _ptr, _ptr, _int]
        L.oracle_sigma.argtypes = [_int, _i64, R, R, _int, _ptr, _ptr, _ptr, _int]
        L.oracle_heat_flux.argtypes = [_int, _i64, R, R, _int, _int, _ptr, _ptr, _ptr, _int]
        L.oracle_totals.argtypes = [_int, _i64, _ptr, _ptr]
        L.oracle_num_threads.argtypes = [_int]
        _libs[prec] = L
    return _libs[prec]


def _p(a: np.ndarray):
    assert a.dtype in (np.float64, np.longdouble) and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ptr)


def _vec(v, D):
    out = np.zeros(3)
    out[:D] = np.asarray(v, dtype=np.float64)[:D]
    return out


def _check(rc, what):
    if rc < 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))
    return rc


# ---------------------------------------------------------------------------
# Lattice and per-cell pieces
# ---------------------------------------------------------------------------

def lattice(lat: int):
    """Return (c (Q,3) int, w (Q,), r, degree) as derived by the oracle."""
    c = np.zeros((64, 3), dtype=np.int32)
    w = np.zeros(64)
    r = _dbl()
    d = _int()
    Q = _check(lib().oracle_lattice(lat, c.ctypes.data_as(_ptr), _p(w), ctypes.byref(r),
                                    ctypes.byref(d)), "lattice")
    return c[:Q].copy(), w[:Q].copy(), r.value, d.value


def velocities(lat: int) -> np.ndarray:
    c, _, r, _ = lattice(lat)
    return r * c[:, :DIM[lat]].astype(np.float64)


def hermite(lat: int, n: int) -> np.ndarray:
    """H^(n)(xi_i) for every velocity, shape (Q,) + (D,)*n."""
    c, _, _, _ = lattice(lat)
    D = DIM[lat]
    out = np.zeros(len(c) * D ** n)
    _check(lib().oracle_hermite(lat, n, _p(out)), "hermite")
    return out.reshape((len(c),) + (D,) * n)


def maxwell_coeff(D: int, n: int, rho: float, u, theta: float) -> np.ndarray:
    out = np.zeros(D ** n)
    _check(lib().oracle_maxwell_coeff(D, n, rho, _p(_vec(u, D)), theta, _p(out)),
           "maxwell_coeff")
    return out.reshape((D,) * n)


def equilibrium(lat: int, rho: float, u, theta: float, eq_order: int = 0) -> np.ndarray:
    Q = len(lattice(lat)[0])
    out = np.zeros(Q)
    _check(lib().oracle_equilibrium(lat, eq_order, rho, _p(_vec(u, DIM[lat])), theta,
                                    _p(out)), "equilibrium")
    return out


def force(lat: int, force_order: int, rho: float, u, theta: float, g, sigma=None) -> np.ndarray:
    D = DIM[lat]
    Q = len(lattice(lat)[0])
    sig = np.zeros(9)
    if sigma is not None:
        sig[:D * D] = np.asarray(sigma, dtype=np.float64).reshape(D * D)
    out = np.zeros(Q)
    _check(lib().oracle_force(lat, force_order, rho, _p(_vec(u, D)), theta, _p(_vec(g, D)),
                              _p(sig), _p(out)), "force")
    return out


# ---------------------------------------------------------------------------
# Force fields
# ---------------------------------------------------------------------------

def g_uniform(D: int, ncell: int, g) -> np.ndarray:
    g = np.asarray(g, dtype=np.float64)[:D]
    return np.ascontiguousarray(np.repeat(g[:, None], ncell, axis=1))


def g_axis_profile(D: int, dims, axis: int, prof) -> np.ndarray:
    """prof: (D, L_axis) acceleration as a function of the coordinate along `axis`
    (0 = x, 1 = y, 2 = z); dims = (nx, ny, nz)."""
    nx, ny, nz = dims
    prof = np.asarray(prof, dtype=np.float64).reshape(D, -1)
    idx = np.indices((nz, ny, nx))  # z, y, x
    coord = idx[2 - axis].reshape(-1)
    return np.ascontiguousarray(prof[:, coord])


# ---------------------------------------------------------------------------
# Simulation
# ---------------------------------------------------------------------------

class OracleSim:
    """A periodic grid of stored populations advanced by the oracle's step."""

    def __init__(self, lat: int, dims, tau_hat: float, rho, u, theta, g,
                 eq_order: int = 0, force_order: int = 4, nthreads: int = 0,
                 prec: str = "f64", mu: float = 0.0, walls=None):
        self.lat = lat
        self.D = DIM[lat]
        self.prec = prec
        self.dt = _DTYPE[prec]
        self.L = lib(prec)
        nx, ny, nz = (tuple(dims) + (1, 1))[:3]
        self.dims = (int(nx), int(ny), int(nz))
        self.N = nx * ny * nz
        self.Q = len(lattice(lat)[0])
        self.tau_hat = float(tau_hat)
        # mu > 0: per-cell relaxation time tau^ = mu/(rho theta) + 1/2 (Sec. 3)
        self.mu = float(mu)
        # walls: None (periodic) or (theta_b, theta_t, U_b, U_t): plates normal to
        # y at y = -1/2 and y = ny - 1/2 (Sec. 3 channel; the wall condition is
        # described in lbm_oracle.c)
        self.walls = None if walls is None else np.asarray(walls, dtype=_DTYPE[prec]).copy()
        self.eq_order = eq_order
        self.force_order = force_order
        self.nthreads = nthreads
        N, D, dt = self.N, self.D, self.dt
        rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dt), (N,)))
        u = np.ascontiguousarray(np.asarray(u, dt).reshape(D, N))
        theta = np.ascontiguousarray(np.broadcast_to(np.asarray(theta, dt), (N,)))
        self.set_force(g)
        self.f = np.zeros((N, self.Q), dtype=dt)
        self._tmp = np.zeros_like(self.f)
        _check(self.L.oracle_init(lat, *self.dims, eq_order, force_order, self._walls_p(),
                                  _p(rho), _p(u), _p(theta), _p(self.g), _p(self.f), nthreads),
               "init")
        self.time = 0

    def set_force(self, g):
        g = np.asarray(g, dtype=np.float64)
        if g.ndim == 1:
            g = g_uniform(self.D, self.N, g)
        self.g = np.ascontiguousarray(g.reshape(self.D, self.N).astype(self.dt))

    def _walls_p(self):
        return None if self.walls is None else _p(self.walls)

    def step(self, n: int = 1):
        _check(self.L.oracle_step(self.lat, *self.dims, self.tau_hat, self.mu, self.eq_order,
                                  self.force_order, self._walls_p(), _p(self.g), _p(self.f),
                                  _p(self._tmp), int(n), self.nthreads), "step")
        self.time += int(n)

    def moments(self):
        """(rho, u, theta) as float64 arrays (rounded from the working precision)."""
        N, D, dt = self.N, self.D, self.dt
        rho, u, th = np.zeros(N, dt), np.zeros((D, N), dt), np.zeros(N, dt)
        _check(self.L.oracle_moments(self.lat, N, _p(self.f), _p(self.g), _p(rho), _p(u),
                                     _p(th), self.nthreads), "moments")
        return rho.astype(np.float64), u.astype(np.float64), th.astype(np.float64)

    def sigma(self):
        N, D = self.N, self.D
        s = np.zeros((D, D, N), self.dt)
        _check(self.L.oracle_sigma(self.lat, N, self.tau_hat, self.mu, self.eq_order, _p(self.f),
                                   _p(self.g), _p(s), self.nthreads), "sigma")
        return s.astype(np.float64)

    def heat_flux(self):
        N, D = self.N, self.D
        q = np.zeros((D, N), self.dt)
        _check(self.L.oracle_heat_flux(self.lat, N, self.tau_hat, self.mu, self.eq_order,
                                       self.force_order, _p(self.f), _p(self.g), _p(q),
                                       self.nthreads), "heat_flux")
        return q.astype(np.float64)

    def totals(self):
        out = np.zeros(2 + self.D, self.dt)
        _check(self.L.oracle_totals(self.lat, self.N, _p(self.f), _p(out)), "totals")
        return out.astype(np.float64)


def num_threads(n: int = 0, prec: str = "f64") -> int:
    return lib(prec).oracle_num_threads(n)
