"""Pins of the finite-difference reference of the channel flow (the paper's
Appendix A), CPU only, against closed forms of the continuum equations of
Sec. 3 (-mu u'' = rho g_x, (rho theta)' = rho g_y, mu u'^2 + lambda theta'' = 0):

* Couette flow (g = 0, moving top plate): u linear and the viscous-heating
  parabola theta = theta_0 + mu U^2 y (H - y) / (2 lambda H^2) are reproduced
  exactly (central differences are exact on quadratics); rho theta uniform.
* Pure conduction with gravity across (g_x = 0): u = 0, theta linear, and the
  density converges to the isothermal barometric law rho ~ exp(g_y y/theta)
  at first order in dy (the forward-difference vertical balance).
* Isothermal, weakly forced Poiseuille flow (g_y = 0): the parabola with peak
  rho_0 g_x H^2 / (8 mu), the paper's U_c.
* Mass: the trapezoidal mean density equals rho_0.
"""
import numpy as np
import pytest

from oracle import fd_poiseuille as fd


def trap_mean(rho):
    return (0.5 * rho[0] + rho[1:-1].sum() + 0.5 * rho[-1]) / (len(rho) - 1)


def test_couette_flow_with_viscous_heating():
    H, N, mu, lam, U, th0 = 10.0, 41, 0.2, 0.4, 0.3, 1.1
    y, rho, u, th, _ = fd.solve(H, N, mu, lam, 0.0, 0.0, 1.0, th0, th0, 0.0, U)
    np.testing.assert_allclose(u, U * y / H, rtol=0, atol=1e-14)
    np.testing.assert_allclose(th, th0 + mu * U * U * y * (H - y) / (2 * lam * H * H),
                               rtol=0, atol=1e-13)
    p = rho * th
    assert np.ptp(p) < 1e-13 * p.mean()
    assert abs(trap_mean(rho) - 1.0) < 1e-14


def test_conduction_with_cross_gravity():
    H, mu, lam, gy = 5.0, 0.1, 0.2, -0.05
    errs = []
    for N in (51, 101, 201):
        y, rho, u, th, _ = fd.solve(H, N, mu, lam, 0.0, gy, 1.0, 1.0, 1.0)
        assert np.abs(u).max() == 0.0
        np.testing.assert_allclose(th, 1.0, rtol=0, atol=1e-13)
        exact = np.exp(gy * y)
        exact *= 1.0 / trap_mean(exact)
        errs.append(np.abs(rho - exact).max())
    assert errs[0] < 1e-3
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2  # first order
    # a temperature difference: theta linear, rho theta obeys the balance
    y, rho, u, th, _ = fd.solve(H, 101, mu, lam, 0.0, gy, 1.0, 0.8, 1.3)
    np.testing.assert_allclose(th, 0.8 + 0.5 * y / H, rtol=0, atol=1e-13)
    dy = y[1] - y[0]
    np.testing.assert_allclose(rho[1:] * th[1:], rho[:-1] * (th[:-1] + gy * dy), rtol=1e-14)
    assert abs(trap_mean(rho) - 1.0) < 1e-14


def test_isothermal_poiseuille_limit():
    H, N, mu, lam = 20.0, 81, 0.5, 1e6  # huge conductivity: no heating
    Uc = 1e-3
    gx = 8 * mu * Uc / H ** 2
    y, rho, u, th, _ = fd.solve(H, N, mu, lam, gx, 0.0, 1.0, 1.0, 1.0)
    np.testing.assert_allclose(u, gx / (2 * mu) * y * (H - y), rtol=0, atol=1e-12 * Uc)
    assert abs(u.max() / Uc - 1.0) < 1e-12


@pytest.mark.parametrize("th_b,th_t", [(1.0, 1.1), (0.7, 1.4)])
def test_paper_channel_converges(th_b, th_t):
    # the channel of Sec. 3: H = 150 lattice spacings, U_c = 1.5, Re = 1800,
    # g_y = -50 g_x, Pr = 1, c_p = 2
    r = 1.1969797703930745
    H = 150 * r
    Uc, Re = 1.5, 1800.0
    mu = Uc * H / Re
    gx = 8 * mu * Uc / H ** 2
    y, rho, u, th, it = fd.solve(H, 601, mu, 2.0 * mu, gx, -50 * gx, 1.0, th_b, th_t)
    assert it < 500
    assert abs(trap_mean(rho) - 1.0) < 1e-13
    assert 0.5 < u.max() < 2.0 and rho.min() > 0.2 and th.min() > 0.5
