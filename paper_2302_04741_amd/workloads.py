"""Seeded synthetic workloads: initial fields and body-force profiles.

This module builds inputs only.  It holds none of the method's arithmetic (no
equilibrium, force term, moments or step): it evaluates the prescribed initial
density, velocity and temperature fields and the force profile on the host in
FP64 and hands the same arrays to whichever solver runs them.

Coordinates are integer node indices x in [0, nx), y in [0, ny), z in [0, nz);
cell = (z*ny + y)*nx + x.  Fields are SoA float64: rho (N,), u (D, N),
theta (N,).  The force is one of
    ("uniform", g)              g: (D,) acceleration per time step,
    ("axis", axis, profile)     profile: (D, L_axis), a function of the
                                coordinate along `axis` (0 = x, 1 = y, 2 = z),
    ("field", g)                g: (D, N).

The three workload families follow the problem statement of the paper (a
periodic compressible fluid with density, velocity and temperature fields,
BGK relaxation time tau-hat and body acceleration g; Sec. 2, eq. (lbm)):
    * ``periodic_2d``     small D2Q37 parity case (64 x 64, constant g);
    * ``thermal_shear_2d`` D2Q37 shear layer with a temperature wave and a
                           transverse gravity (1024 x 1024 by default);
    * ``kolmogorov_3d``   D3Q39 Kolmogorov-forced flow with a temperature wave
                           and a seeded random-phase velocity perturbation
                           (256^3 by default).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import numpy as np

LATTICE_DIM = {"D2Q37": 2, "D3Q39": 3}
# lattice spacing r of each velocity set (velocities are r times integer vectors)
LATTICE_R = {"D2Q37": 1.1969797703930745, "D3Q39": math.sqrt(1.5)}

#: seed of the random phases of the 3-D velocity perturbation
KOLMOGOROV_SEED = 230204741


@dataclasses.dataclass
class Workload:
    name: str
    lattice: str
    dims: Tuple[int, int, int]
    tau_hat: float
    rho: np.ndarray
    u: np.ndarray
    theta: np.ndarray
    force: tuple
    steps: int
    eq_order: int = 0
    force_order: int = 4
    mu: float = 0.0  # > 0: per-cell relaxation time tau^ = mu/(rho theta) + 1/2
    walls: tuple | None = None  # (theta_b, theta_t, U_b, U_t): plates normal to y

    @property
    def D(self) -> int:
        return LATTICE_DIM[self.lattice]

    @property
    def ncell(self) -> int:
        nx, ny, nz = self.dims
        return nx * ny * nz

    def force_field(self) -> np.ndarray:
        """The force as a full (D, N) float64 field (any kind)."""
        D, N = self.D, self.ncell
        kind = self.force[0]
        if kind == "uniform":
            g = np.asarray(self.force[1], dtype=np.float64)[:D]
            return np.ascontiguousarray(np.repeat(g[:, None], N, axis=1))
        if kind == "axis":
            axis, prof = self.force[1], np.asarray(self.force[2], dtype=np.float64)
            nx, ny, nz = self.dims
            coord = np.indices((nz, ny, nx))[2 - axis].reshape(-1)
            return np.ascontiguousarray(prof.reshape(D, -1)[:, coord])
        if kind == "field":
            return np.ascontiguousarray(np.asarray(self.force[1], np.float64).reshape(D, N))
        raise ValueError("unknown force kind %r" % (kind,))


def _grid(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def periodic_2d(n: int = 64, tau_hat: float = 0.8, g=(1e-5, 0.0), steps: int = 1000,
                force_order: int = 4) -> Workload:
    """rho = 1 + 0.01 sin(2 pi x/n), theta = 1 + 0.05 sin(2 pi y/n), u = 0."""
    dims = (n, n, 1)
    x, y, _ = _grid(dims)
    rho = 1.0 + 0.01 * np.sin(2.0 * math.pi * x / n)
    theta = 1.0 + 0.05 * np.sin(2.0 * math.pi * y / n)
    u = np.zeros((2, n * n))
    return Workload("D2Q37 %dx%d periodic, uniform g" % (n, n), "D2Q37", dims, tau_hat,
                    rho, u, theta, ("uniform", np.asarray(g, np.float64)), steps,
                    force_order=force_order)


def thermal_shear_2d(n: int = 1024, tau_hat: float = 0.6, dtheta: float = 0.02,
                     mach: float = 0.05, g=(0.0, -1e-5), steps: int = 5000,
                     force_order: int = 4, ny: int | None = None) -> Workload:
    """theta = 1 + dtheta sin(2 pi y/L), u_x = Ma sqrt(theta) sin(2 pi y/L),
    u_y = 0, rho = 1, uniform g (transverse by default)."""
    ny = n if ny is None else ny
    dims = (n, ny, 1)
    _, y, _ = _grid(dims)
    s = np.sin(2.0 * math.pi * y / ny)
    theta = 1.0 + dtheta * s
    u = np.zeros((2, n * ny))
    u[0] = mach * np.sqrt(theta) * s
    rho = np.ones(n * ny)
    name = "D2Q37 %dx%d shear, tau=%g dtheta=%g Ma=%g" % (n, ny, tau_hat, dtheta, mach)
    return Workload(name, "D2Q37", dims, tau_hat, rho, u, theta,
                    ("uniform", np.asarray(g, np.float64)), steps, force_order=force_order)


def channel(theta_b: float = 0.7, theta_t: float = 1.4, nx: int = 3, ny: int = 150,
            u_c: float = 1.5, re: float = 1800.0, steps: int = 150_000,
            force_order: int = 4) -> Workload:
    """The channel of Sec. 3: D2Q37 between plates at rest (height H = ny r),
    dynamic viscosity mu = rho0 U_c H / Re held constant by the per-cell
    relaxation time, g_x = 8 mu U_c / (rho0 H^2) along the channel and
    g_y = -50 g_x across it (rho0 = 1).  Starts from rest at uniform density
    with theta linear between the plate temperatures."""
    H = ny * LATTICE_R["D2Q37"]
    mu = u_c * H / re
    gx = 8.0 * mu * u_c / H ** 2
    dims = (nx, ny, 1)
    _, y, _ = _grid(dims)
    theta = theta_b + (theta_t - theta_b) * (y + 0.5) / ny
    name = "D2Q37 %dx%d channel, plates %g/%g" % (nx, ny, theta_b, theta_t)
    return Workload(name, "D2Q37", dims, 0.8, np.ones(nx * ny), np.zeros((2, nx * ny)), theta,
                    ("uniform", np.array([gx, -50.0 * gx])), steps, force_order=force_order,
                    mu=mu, walls=(theta_b, theta_t, 0.0, 0.0))


def kolmogorov_modes():
    """The 62 integer wave vectors k with 1 <= |k|_inf <= 2 whose first nonzero
    component is positive (one of each +-k pair)."""
    ks = []
    for kx in range(-2, 3):
        for ky in range(-2, 3):
            for kz in range(-2, 3):
                k = (kx, ky, kz)
                if k == (0, 0, 0):
                    continue
                first = next(c for c in k if c != 0)
                if first > 0:
                    ks.append(k)
    return np.asarray(ks, dtype=np.int64)


def kolmogorov_3d(n: int = 256, tau_hat: float = 0.8, g0: float = 1e-5, amp: float = 1e-3,
                  seed: int = KOLMOGOROV_SEED, steps: int = 2000,
                  force_order: int = 4) -> Workload:
    """rho = 1, theta = 1 + 0.05 sin(2 pi y/n), Kolmogorov force
    g_x = g0 sin(2 pi z/n) along z, and u_a = A sum_k sin(2 pi k.x/n + phi_ak)
    over the 62 modes of ``kolmogorov_modes`` with phases drawn from
    default_rng(seed).uniform(0, 2 pi, (3, 62)) and A = amp sqrt(2/62), so that
    each component has RMS ``amp``."""
    dims = (n, n, n)
    N = n ** 3
    ks = kolmogorov_modes()
    phi = np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, (3, len(ks)))
    A = amp * math.sqrt(2.0 / len(ks))
    u = np.empty((3, N))
    # sin(2 pi k.x/n + phi) summed via the inverse FFT of a spectrum holding
    # exp(i phi)/(2i) at k and its conjugate at -k.
    for a in range(3):
        spec = np.zeros((n, n, n), dtype=np.complex128)  # axes (z, y, x)
        for m, (kx, ky, kz) in enumerate(ks):
            c = np.exp(1j * phi[a, m]) / 2j
            spec[kz % n, ky % n, kx % n] += c
            spec[(-kz) % n, (-ky) % n, (-kx) % n] += np.conj(c)
        field = np.fft.ifftn(spec).real * float(N)
        u[a] = A * field.reshape(-1)
        del spec, field
    _, y, _ = _grid(dims)
    theta = 1.0 + 0.05 * np.sin(2.0 * math.pi * y / n)
    rho = np.ones(N)
    prof = np.zeros((3, n))
    prof[0] = g0 * np.sin(2.0 * math.pi * np.arange(n) / n)
    name = "D3Q39 %d^3 Kolmogorov" % n
    return Workload(name, "D3Q39", dims, tau_hat, rho, u, theta, ("axis", 2, prof), steps,
                    force_order=force_order)


def random_smooth(lattice: str, dims, seed: int, tau_hat: float = 0.7, amp_u: float = 0.05,
                  amp_rho: float = 0.02, amp_theta: float = 0.05, g_amp: float = 1e-4,
                  force_kind: str = "uniform", steps: int = 10,
                  force_order: int = 4) -> Workload:
    """Smooth random fields for edge-case tests: a few low Fourier modes with
    seeded amplitudes and phases on any (possibly ragged) periodic grid."""
    D = LATTICE_DIM[lattice]
    nx, ny, nz = dims
    if D == 2 and nz != 1:
        raise ValueError("2-D lattice needs nz == 1")
    rng = np.random.default_rng(seed)
    x, y, z = _grid(dims)

    def smooth(amp):
        out = np.zeros(x.shape)
        for _ in range(3):
            kx, ky, kz = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            arg = 2 * math.pi * (kx * x / nx + ky * y / ny + (kz * z / nz if D == 3 else 0.0))
            out += rng.uniform(-1, 1) * np.sin(arg + ph)
        return amp * out / 3.0

    rho = 1.0 + smooth(amp_rho)
    theta = 1.0 + smooth(amp_theta)
    u = np.stack([smooth(amp_u) for _ in range(D)])
    g = rng.uniform(-1, 1, size=D) * g_amp
    if force_kind == "uniform":
        force = ("uniform", g)
    elif force_kind == "axis":
        axis = int(rng.integers(0, D))
        L = dims[axis]
        prof = np.outer(g, np.sin(2 * math.pi * np.arange(L) / L + rng.uniform(0, 6.28)))
        force = ("axis", axis, prof)
    elif force_kind == "field":
        force = ("field", np.stack([g[a] * (1.0 + smooth(0.5)) for a in range(D)]))
    else:
        raise ValueError(force_kind)
    return Workload("%s %s random seed %d" % (lattice, "x".join(map(str, dims)), seed),
                    lattice, tuple(dims), tau_hat, rho, u, theta, force, steps,
                    force_order=force_order)
