"""Finite-difference reference of the steady compressible Poiseuille flow with
cross-flow gravity (the paper's Appendix A; the flow of Sec. 3).

TEST INFRASTRUCTURE ONLY (part of the oracle): only the test suite may use it.

The steady, x-independent flow between plates at y = 0 and y = H with u = u_x(y),
u_y = 0 obeys (Sec. 3)
    -mu u'' = rho g_x,   (rho theta)' = rho g_y,   mu (u')^2 + lambda theta'' = 0,
with u, theta given at both plates and the mean density rho_0.  On N nodes
y_j = (j - 1) dy, dy = H/(N - 1), the appendix discretises the momentum and
energy equations with central differences and the vertical balance with a
forward difference, closes the system with the trapezoidal mass constraint
    rho_1/2 + rho_2 + ... + rho_{N-1} + rho_N/2 = rho_0 (N - 1),
and solves it by a fixed-point iteration that lags the viscous-heating term:
temperature from the energy equation, then density from the vertical balance
and the mass constraint, then velocity from the momentum equation.  The first
velocity guess is the incompressible profile with the plate velocities.
"""
from __future__ import annotations

import numpy as np


def _tridiag_dirichlet(rhs_inner, left, right):
    """Solve v_{j+1} - 2 v_j + v_{j-1} = rhs_j for the inner nodes j = 2..N-1
    with v_1 = left, v_N = right (a plain tridiagonal solve)."""
    n = len(rhs_inner)
    a = np.diag(-2.0 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    b = np.array(rhs_inner, dtype=np.float64)
    b[0] -= left
    b[-1] -= right
    return np.concatenate([[left], np.linalg.solve(a, b), [right]])


def solve(H: float, N: int, mu: float, lam: float, gx: float, gy: float, rho0: float,
          theta_b: float, theta_t: float, u_b: float = 0.0, u_t: float = 0.0,
          tol: float = 1e-13, max_iter: int = 10000):
    """Return (y, rho, u, theta) on the N nodes, and the iteration count."""
    y = np.linspace(0.0, H, N)
    dy = H / (N - 1)
    u = -gx / (2.0 * mu) * y * (y - H) + (u_t - u_b) / H * y + u_b
    for it in range(1, max_iter + 1):
        # energy: 4 lambda (theta_{j+1} - 2 theta_j + theta_{j-1}) = -mu (u_{j+1} - u_{j-1})^2
        heat = -mu * (u[2:] - u[:-2]) ** 2 / (4.0 * lam)
        theta = _tridiag_dirichlet(heat, theta_b, theta_t)
        # vertical balance: rho_{j+1} theta_{j+1} = rho_j (theta_j + g_y dy)
        ratio = (theta[:-1] + gy * dy) / theta[1:]
        shape = np.concatenate([[1.0], np.cumprod(ratio)])
        mass = 0.5 * shape[0] + shape[1:-1].sum() + 0.5 * shape[-1]
        rho = shape * rho0 * (N - 1) / mass
        # momentum: u_{j+1} - 2 u_j + u_{j-1} = -(g_x dy^2 / mu) rho_j
        u_new = _tridiag_dirichlet(-gx * dy * dy / mu * rho[1:-1], u_b, u_t)
        change = np.abs(u_new - u).max()
        u = u_new
        if change <= tol * max(1.0, np.abs(u).max()):
            # one more temperature/density pass with the converged velocity
            heat = -mu * (u[2:] - u[:-2]) ** 2 / (4.0 * lam)
            theta = _tridiag_dirichlet(heat, theta_b, theta_t)
            ratio = (theta[:-1] + gy * dy) / theta[1:]
            shape = np.concatenate([[1.0], np.cumprod(ratio)])
            mass = 0.5 * shape[0] + shape[1:-1].sum() + 0.5 * shape[-1]
            rho = shape * rho0 * (N - 1) / mass
            return y, rho, u, theta, it
    raise RuntimeError("finite-difference iteration did not converge")
