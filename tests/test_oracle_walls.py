"""Pins of the oracle's plates (CPU only).  The paper runs its channel flow
(Sec. 3) between two plates with a wall condition it does not publish; the
oracle's plates are this project's diffuse-reflection design with the absorbed
mass re-emitted per column.  Pinned by what any consistent wall must satisfy:

* mass is conserved exactly (force and plates included), momentum is not;
* a gas at rest at the plates' temperature stays exactly at rest;
* Couette flow between plates moving at -U and +U is linear and antisymmetric,
  with a slope within a few per cent of 2U/H (kinetic slip);
* steady conduction between plates at different temperatures: theta linear
  outside a Knudsen layer of three nodes at each plate, pressure uniform, no
  flow;
* isothermal Poiseuille flow matches the finite-difference reference of the
  paper's Appendix A (here the parabola), with a slip excess that halves when
  the channel height doubles (first order in the Knudsen number).
"""
import numpy as np

from oracle import fd_poiseuille as fd


def channel(oracle_mod, ny, walls, tau=0.8, g=(0.0, 0.0), theta=1.0, nx=1, u=None, mu=0.0):
    N = nx * ny
    u = np.zeros((2, N)) if u is None else u
    gg = np.zeros((2, N))
    gg[0], gg[1] = g
    return oracle_mod.OracleSim(0, (nx, ny, 1), tau, 1.0, u, theta, gg, walls=walls, mu=mu)


def test_mass_conserved_momentum_not(oracle_mod):
    rng = np.random.default_rng(0)
    nx, ny = 3, 20
    N = nx * ny
    u = rng.uniform(-0.05, 0.05, (2, N))
    theta = 1 + rng.uniform(-0.05, 0.05, N)
    rho = 1 + rng.uniform(-0.02, 0.02, N)
    g = np.zeros((2, N))
    g[0], g[1] = 1e-4, -2e-4
    s = oracle_mod.OracleSim(0, (nx, ny, 1), 0.7, rho, u, theta, g,
                             walls=(0.9, 1.2, 0.02, -0.03))
    t0 = s.totals()
    s.step(50)
    t1 = s.totals()
    assert abs(t1[0] / t0[0] - 1) < 1e-13
    assert abs(t1[2] - t0[2]) > 1e-4 * abs(t0[0])  # the plates exert a force


def test_gas_at_rest_stays_at_rest(oracle_mod):
    s = oracle_mod.OracleSim(0, (2, 12, 1), 0.8, 1.1, np.zeros((2, 24)), 0.9, np.zeros((2, 24)),
                             walls=(0.9, 0.9, 0.0, 0.0))
    f0 = s.f.copy()
    s.step(30)
    assert np.abs(s.f - f0).max() < 1e-14


def test_couette_flow(oracle_mod):
    r = oracle_mod.lattice(0)[2]
    ny, U = 40, 0.01
    s = channel(oracle_mod, ny, (1.0, 1.0, -U, U))
    s.step(20000)
    _, u, _ = s.moments()
    y = (np.arange(ny) + 0.5) * r
    H = ny * r
    p = np.polyfit(y, u[0], 1)
    assert abs(np.polyval(p, H / 2)) < 1e-12 * U
    np.testing.assert_allclose(u[0], -u[0][::-1], rtol=0, atol=1e-13)
    assert np.abs(u[0] - np.polyval(p, y)).max() < 5e-3 * U
    assert 0.97 < p[0] / (2 * U / H) < 1.0
    assert np.abs(u[1]).max() < 1e-5 * U


def test_steady_conduction(oracle_mod):
    r = oracle_mod.lattice(0)[2]
    ny = 40
    s = channel(oracle_mod, ny, (0.95, 1.05, 0.0, 0.0))
    s.step(20000)
    rho, u, th = s.moments()
    y = (np.arange(ny) + 0.5) * r
    H = ny * r
    p = np.polyfit(y[3:-3], th[3:-3], 1)
    res = np.abs(th - np.polyval(p, y))
    assert res[3:-3].max() < 1e-3 * 0.1  # linear away from the plates
    assert res.max() < 5e-3 * 0.1  # a thin Knudsen layer at the plates
    assert 0.96 < p[0] / (0.1 / H) < 1.0
    pr = rho * th
    assert pr.std() < 2e-4 * pr.mean()
    assert np.abs(u).max() < 1e-3 * 0.1


def test_isothermal_poiseuille_against_finite_difference(oracle_mod):
    r = oracle_mod.lattice(0)[2]
    tau, gx = 0.8, 1e-6
    excess = []
    for ny, steps in ((30, 15000), (60, 45000)):
        H = ny * r
        s = channel(oracle_mod, ny, (1.0, 1.0, 0.0, 0.0), tau=tau, g=(gx, 0.0))
        s.step(steps)
        _, u, _ = s.moments()
        mu = tau - 0.5  # nu = (tau^ - 1/2) theta at rho = theta = 1
        yf, _, uf, _, _ = fd.solve(H, 10 * ny + 1, mu, 2 * mu, gx, 0.0, 1.0, 1.0, 1.0)
        ref = np.interp((np.arange(ny) + 0.5) * r, yf, uf)
        excess.append(u[0].max() / ref.max() - 1)
        # the same parabola up to the slip, which is uniform across the channel
        shape = (u[0] - u[0].min()) / (ref - ref.min()).max()
        assert np.abs(shape - (ref - ref.min()) / (ref - ref.min()).max()).max() < 2e-2
    assert 0.0 < excess[0] < 0.06
    assert 1.8 < excess[0] / excess[1] < 2.2
