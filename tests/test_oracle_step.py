"""Pins of the oracle's time step, eq. (lbm) of the paper (CPU only).

* Chapman-Enskog contraction behind q_err (Sec. 2): the printed closed form
  equals (1/12) a_1^(3) : int omega H^(3) c^2 c with a_1^(3) = -3 tau g a_0^(2).
* Uniform fluid under constant g: rho and theta constant, u(n) = u0 + n g.
* Global invariants on a ragged periodic grid: mass constant, momentum grows by
  sum rho g and energy by sum 2 rho g.u per step (moments of eq. (F) with
  eq. (lbm)).
* Shear-wave decay at nu = (tau-hat - 1/2) theta (tau = tau-hat - 1/2, Sec. 2),
  with second-order convergence of the lattice error.
* Isobaric temperature wave (the entropy mode) decaying at the thermal
  diffusivity lambda/(rho c_p) = nu: BGK has Prandtl number 1.
* Isentropic standing sound wave oscillating at the adiabatic speed of sound
  sqrt(gamma theta), gamma = (D + 2)/D (an isothermal model would give
  sqrt(theta)), with second-order convergence of the lattice error.
* Mid-point stress sigma-bar against the Newtonian stress of the Chapman-Enskog
  estimate (Sec. 2): sigma = mu (grad u + grad u^T - (2/D) div u delta).
* The paper's central claim (abstract, Sec. 2): dropping the third-moment force
  term changes the heat flux by q_err.
* Initial state reproduces the input moments; results do not depend on the
  number of threads.
* Per-cell relaxation time tau = mu/(rho theta) (Sec. 3, used there to keep the
  dynamic viscosity constant): the shear-wave rate is mu/rho at any temperature;
  in a gas whose pressure varies by +-15% the local stress is mu grad u at every
  cell (while the constant-tau scheme gives (tau-hat - 1/2) p grad u); a
  uniform state reduces to the constant-tau run with tau-hat = mu/(rho theta)
  + 1/2; q_err holds with tau = mu/(rho theta).
"""

import numpy as np
import pytest

from _ref import explicit_hermite, maxwellian_average
from paper_2302_04741_amd import workloads


def q_err_printed(D, rho, u, theta, g, tau):
    u, g = np.asarray(u), np.asarray(g)
    return -0.5 * rho * tau * ((u @ u + (theta - 1.0) * (D + 2)) * g + 2.0 * (g @ u) * u)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chapman_enskog_contraction(D, seed):
    rng = np.random.default_rng(seed)
    rho, theta, tau = rng.uniform(0.8, 1.2), rng.uniform(0.7, 1.4), rng.uniform(0.1, 0.6)
    u, g = rng.normal(size=D) * 0.2, rng.normal(size=D) * 1e-3
    a02 = rho * (np.outer(u, u) + (theta - 1.0) * np.eye(D))
    a13 = -tau * (np.einsum("a,bc->abc", g, a02) + np.einsum("b,ac->abc", g, a02)
                  + np.einsum("c,ab->abc", g, a02))

    def integrand(xi):
        c = xi - u
        return np.multiply.outer(explicit_hermite(xi, 3), (c @ c) * c)

    # integral of omega(xi) H3(xi) c^2 c: Gaussian weight with rho=1, u=0, theta=1
    M = maxwellian_average(D, 1.0, np.zeros(D), 1.0, integrand, npts=6)
    q = np.einsum("abc,abcd->d", a13, M) / 12.0
    np.testing.assert_allclose(q, q_err_printed(D, rho, u, theta, g, tau), rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_uniform_fluid_accelerates_exactly(oracle_mod, lat, order):
    D = oracle_mod.DIM[lat]
    u0 = np.array([0.05, -0.03, 0.02][:D])
    g = np.array([1e-5, -2e-5, 3e-5][:D])
    sim = oracle_mod.OracleSim(lat, (1, 1, 1), 0.8, 1.0, u0.reshape(D, 1), 1.1, g,
                               force_order=order)
    r, u, t = sim.moments()
    assert abs(r[0] - 1.0) < 1e-15 and abs(t[0] - 1.1) < 1e-15
    np.testing.assert_allclose(u[:, 0], u0, atol=1e-16)
    for n in (1, 10, 200):
        sim.step(n - sim.time)
        r, u, t = sim.moments()
        assert abs(r[0] - 1.0) < 2e-14
        assert abs(t[0] - 1.1) < 2e-13
        np.testing.assert_allclose(u[:, 0], u0 + n * g, rtol=0, atol=1e-14)


@pytest.mark.parametrize("lat,dims", [(0, (13, 10, 1)), (1, (7, 5, 6))])
def test_global_invariants_ragged_grid(oracle_mod, lat, dims):
    name = "D2Q37" if lat == 0 else "D3Q39"
    wl = workloads.random_smooth(name, dims, seed=5, force_kind="field", g_amp=1e-3)
    g = wl.force_field()
    sim = oracle_mod.OracleSim(lat, dims, wl.tau_hat, wl.rho, wl.u, wl.theta, g)
    D = oracle_mod.DIM[lat]
    for _ in range(5):
        tot0 = sim.totals()
        rho, u, _ = sim.moments()
        sim.step(1)
        tot1 = sim.totals()
        assert abs(tot1[0] - tot0[0]) < 1e-12 * tot0[0]
        dmom = (rho[None, :] * g).sum(axis=1)
        np.testing.assert_allclose(tot1[1:1 + D] - tot0[1:1 + D], dmom, rtol=0,
                                   atol=1e-13 * tot0[0])
        de = 2.0 * (rho * (g * u).sum(axis=0)).sum()
        # rounding of a sum of N*Q terms of size ~|total|: 1e-13 relative to the total
        assert abs((tot1[1 + D] - tot0[1 + D]) - de) < 1e-13 * tot0[1 + D]


def shear_wave_rate(oracle_mod, lat, L, tau_hat, theta=1.0, rho=1.0, mu=0.0):
    D = oracle_mod.DIM[lat]
    y = np.arange(L)
    s = np.sin(2 * np.pi * y / L)
    u = np.zeros((D, L))
    u[0] = 1e-4 * s
    dims = (1, L, 1)
    sim = oracle_mod.OracleSim(lat, dims, tau_hat, rho, u, theta, np.zeros(D), mu=mu)
    sim.step(200)  # let the initial non-equilibrium transient decay
    amps = []
    for _ in range(3):
        amps.append(2.0 / L * (sim.moments()[1][0] * s).sum())
        sim.step(200)
    return -np.log(amps[-1] / amps[0]) / 400.0


@pytest.mark.parametrize("lat", [0, 1])
def test_shear_wave_viscosity(oracle_mod, lat):
    tau_hat, theta = 0.8, 1.0
    r = oracle_mod.lattice(lat)[2]
    errs = []
    for L in (32, 64):
        k = 2 * np.pi / L / r  # wavenumber per unit length; the lattice spacing is r
        nu = (tau_hat - 0.5) * theta
        errs.append(shear_wave_rate(oracle_mod, lat, L, tau_hat, theta) / (nu * k * k) - 1.0)
    assert abs(errs[1]) < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0  # O(k^2) lattice error


def test_shear_wave_viscosity_depends_on_theta(oracle_mod):
    r = oracle_mod.lattice(0)[2]
    L, tau_hat, theta = 64, 0.9, 1.3
    k = 2 * np.pi / L / r
    rate = shear_wave_rate(oracle_mod, 0, L, tau_hat, theta)
    assert abs(rate / ((tau_hat - 0.5) * theta * k * k) - 1.0) < 3e-3


@pytest.mark.parametrize("lat", [0, 1])
def test_sigma_is_newtonian_stress(oracle_mod, lat):
    D = oracle_mod.DIM[lat]
    L, tau_hat = 64, 0.8
    r = oracle_mod.lattice(lat)[2]
    y = np.arange(L)
    s, c = np.sin(2 * np.pi * y / L), np.cos(2 * np.pi * y / L)
    u = np.zeros((D, L))
    u[0] = 1e-4 * s
    sim = oracle_mod.OracleSim(lat, (1, L, 1), tau_hat, 1.0, u, 1.0, np.zeros(D))
    sim.step(100)
    ux = sim.moments()[1][0]
    sig = sim.sigma()
    a_u = 2.0 / L * (ux * s).sum()
    a_s = 2.0 / L * (sig[0, 1] * c).sum()
    mu = (tau_hat - 0.5) * 1.0 * 1.0
    expected = mu * a_u * (2 * np.pi / L) / r  # d/dy of a_u sin(k j), j = y / r
    assert abs(a_s / expected - 1.0) < 5e-3
    assert np.abs(sig[0, 0]).max() < 1e-3 * abs(a_s)  # no normal stress in a pure shear


@pytest.mark.parametrize("lat", [0, 1])
def test_dropping_a3F_adds_chapman_enskog_heat_flux(oracle_mod, lat):
    D = oracle_mod.DIM[lat]
    tau_hat = 0.8
    u0 = np.array([0.1, 0.05, -0.04][:D])
    g = np.array([1e-5, -2e-5, 1.5e-5][:D])
    q = {}
    for order in (2, 4):
        sim = oracle_mod.OracleSim(lat, (1, 1, 1), tau_hat, 1.0, u0.reshape(D, 1), 1.2, g,
                                   force_order=order)
        sim.step(60)
        q[order] = sim.heat_flux()[:, 0]
        rho, u, theta = sim.moments()
    dq = q[2] - q[4]
    ref = q_err_printed(D, rho[0], u[:, 0], theta[0], g, tau_hat - 0.5)
    np.testing.assert_allclose(dq, ref, rtol=1e-4, atol=0)
    # with the full scheme the heat flux of a uniform flow is O(g^2), far below q_err
    assert np.abs(q[4]).max() < 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("lat,dims", [(0, (9, 11, 1)), (1, (5, 4, 6))])
@pytest.mark.parametrize("order", [2, 3, 4])
def test_initial_state_reproduces_inputs(oracle_mod, lat, dims, order):
    name = "D2Q37" if lat == 0 else "D3Q39"
    wl = workloads.random_smooth(name, dims, seed=3, force_kind="field", g_amp=1e-3)
    sim = oracle_mod.OracleSim(lat, dims, wl.tau_hat, wl.rho, wl.u, wl.theta, wl.force_field(),
                               force_order=order)
    r, u, t = sim.moments()
    np.testing.assert_allclose(r, wl.rho, rtol=0, atol=1e-15)
    np.testing.assert_allclose(u, wl.u, rtol=0, atol=1e-15)
    np.testing.assert_allclose(t, wl.theta, rtol=0, atol=2e-15)


def test_thread_count_does_not_change_results(oracle_mod):
    wl = workloads.random_smooth("D3Q39", (6, 7, 5), seed=9, force_kind="axis")
    out = []
    for nt in (1, 4):
        sim = oracle_mod.OracleSim(1, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta,
                                   wl.force_field(), nthreads=nt)
        sim.step(3)
        out.append(sim.f.copy())
    assert np.array_equal(out[0], out[1])


def test_parity_workload_runs_stably(oracle_mod):
    wl = workloads.periodic_2d()
    sim = oracle_mod.OracleSim(0, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta, wl.force_field())
    m0 = sim.totals()[0]
    sim.step(200)
    r, u, t = sim.moments()
    assert np.all(np.isfinite(r)) and np.all(np.isfinite(t))
    assert abs(sim.totals()[0] - m0) < 1e-12 * m0
    # the uniform force accelerates the mean flow: sum rho u grows by n * sum rho g
    np.testing.assert_allclose((r * u[0]).sum(), 200 * 1e-5 * m0, rtol=1e-9)


@pytest.mark.parametrize("lat,theta,rho", [(0, 0.8, 1.0), (0, 1.3, 1.0), (0, 1.0, 1.25),
                                           (1, 1.3, 1.0)])
def test_viscosity_mode_shear_wave_rate_is_mu_over_rho(oracle_mod, lat, theta, rho):
    mu, L = 0.35, 64
    r = oracle_mod.lattice(lat)[2]
    k = 2 * np.pi / L / r
    # tau_hat is ignored when mu > 0
    rate = shear_wave_rate(oracle_mod, lat, L, 0.0, theta, rho, mu)
    assert abs(rate / (mu / rho * k * k) - 1.0) < 3e-3


@pytest.mark.parametrize("lat", [0, 1])
def test_viscosity_mode_uniform_state_reduces_to_constant_tau(oracle_mod, lat):
    D = oracle_mod.DIM[lat]
    rho0, th0, mu = 1.2, 0.9, 0.4
    u0 = np.array([0.05, -0.03, 0.02][:D]).reshape(D, 1)
    g = np.array([1e-5, -2e-5, 3e-5][:D])
    a = oracle_mod.OracleSim(lat, (1, 1, 1), 0.0, rho0, u0, th0, g, mu=mu)
    b = oracle_mod.OracleSim(lat, (1, 1, 1), mu / (rho0 * th0) + 0.5, rho0, u0, th0, g)
    a.step(50)
    b.step(50)
    np.testing.assert_allclose(a.f, b.f, rtol=0, atol=1e-14)
    np.testing.assert_allclose(a.heat_flux(), b.heat_flux(), rtol=1e-10, atol=1e-18)


def test_viscosity_mode_stress_is_mu_grad_u_where_pressure_varies(oracle_mod):
    """1-D gas with theta = 1 + 0.2 sin(2 pi x / 64) at rho = 1 (pressure varies
    +-15% and oscillates acoustically) carrying a transverse shear u_y(x).  The
    local Newtonian law sigma_xy = mu du_y/dx must hold at every cell with the
    constant mu; with a constant tau-hat it holds with (tau-hat - 1/2) p(x)."""
    lat, D, L = 0, 2, 64
    r = oracle_mod.lattice(lat)[2]
    x = np.arange(L)
    theta = 1 + 0.2 * np.sin(2 * np.pi * x / L)
    u = np.zeros((D, L))
    u[1] = 1e-4 * np.sin(2 * np.pi * 2 * x / L)
    kk = 2 * np.pi * np.fft.fftfreq(L) / r  # the lattice spacing is r

    def ddx(f):
        return np.real(np.fft.ifft(1j * kk * np.fft.fft(f)))

    mu, tau_hat = 0.3, 0.8
    for n in (5, 20, 60):
        out = {}
        for mode in ("mu", "tau"):
            sim = oracle_mod.OracleSim(lat, (L, 1, 1), tau_hat, 1.0, u, theta, np.zeros(D),
                                       mu=mu if mode == "mu" else 0.0)
            sim.step(n)
            rho, uu, th = sim.moments()
            du = ddx(uu[1])
            sel = np.abs(du) > 0.5 * np.abs(du).max()
            out[mode] = (sim.sigma()[0, 1][sel] / du[sel], (rho * th)[sel])
        ratio, p = out["mu"]
        assert p.max() / p.min() > 1.15
        assert np.abs(ratio / mu - 1).max() < 1.5e-2
        ratio_t, p_t = out["tau"]
        assert np.abs(ratio_t / ((tau_hat - 0.5) * p_t) - 1).max() < 1.5e-2
        # the two schemes differ by the local pressure
        assert np.abs(ratio_t / (tau_hat - 0.5) - ratio / mu).max() > 0.1


@pytest.mark.parametrize("lat", [0, 1])
def test_viscosity_mode_q_err(oracle_mod, lat):
    D = oracle_mod.DIM[lat]
    mu = 0.25
    u0 = np.array([0.1, 0.05, -0.04][:D])
    g = np.array([1e-5, -2e-5, 1.5e-5][:D])
    q = {}
    for order in (2, 4):
        sim = oracle_mod.OracleSim(lat, (1, 1, 1), 0.0, 1.1, u0.reshape(D, 1), 1.2, g,
                                   force_order=order, mu=mu)
        sim.step(60)
        q[order] = sim.heat_flux()[:, 0]
        rho, u, theta = sim.moments()
    ref = q_err_printed(D, rho[0], u[:, 0], theta[0], g, mu / (rho[0] * theta[0]))
    np.testing.assert_allclose(q[2] - q[4], ref, rtol=1e-4, atol=0)


def temperature_wave_rate(oracle_mod, lat, L, tau_hat):
    """Decay rate of theta = 1 + eps sin(2 pi y/L) at uniform pressure (rho =
    1/theta, u = 0), from a least-squares fit of log(amplitude) over one e-fold
    of the expected decay (averages out the weak sound waves of the start)."""
    D = oracle_mod.DIM[lat]
    r = oracle_mod.lattice(lat)[2]
    y = np.arange(L)
    s = np.sin(2 * np.pi * y / L)
    theta = 1 + 1e-4 * s
    sim = oracle_mod.OracleSim(lat, (1, L, 1), tau_hat, 1 / theta, np.zeros((D, L)), theta,
                               np.zeros(D))
    k = 2 * np.pi / L / r
    e_fold = 1 / ((tau_hat - 0.5) * k * k)
    n0, n1 = int(0.3 * e_fold), int(1.3 * e_fold)
    ts, amps = [], []
    for n in range(n0, n1, max(1, (n1 - n0) // 100)):
        sim.step(n - sim.time)
        th = sim.moments()[2]
        ts.append(n)
        amps.append(2.0 / L * ((th - 1) * s).sum())
    return -np.polyfit(ts, np.log(amps), 1)[0], k


@pytest.mark.parametrize("lat", [0, 1])
def test_temperature_wave_decays_at_nu(oracle_mod, lat):
    tau_hat = 0.8
    errs = []
    for L in (32, 64):
        rate, k = temperature_wave_rate(oracle_mod, lat, L, tau_hat)
        errs.append(abs(rate / ((tau_hat - 0.5) * k * k) - 1))
    assert errs[1] < 4e-3
    assert errs[1] < errs[0]  # the lattice error shrinks with the wavelength


def sound_frequency_ratio(oracle_mod, lat, L):
    """omega / (c_s k) of an isentropic standing wave (rho and theta in phase,
    delta theta/theta = (gamma - 1) delta rho/rho, u = 0), from the zero
    crossings of the density amplitude over four periods."""
    D = oracle_mod.DIM[lat]
    r = oracle_mod.lattice(lat)[2]
    gamma = (D + 2) / D
    y = np.arange(L)
    s = np.sin(2 * np.pi * y / L)
    rho = 1 + 1e-4 * s
    theta = 1 + (gamma - 1) * 1e-4 * s
    sim = oracle_mod.OracleSim(lat, (1, L, 1), 0.8, rho, np.zeros((D, L)), theta, np.zeros(D))
    k = 2 * np.pi / L / r
    period = 2 * np.pi / (np.sqrt(gamma) * k)
    a = []
    for _ in range(int(4 * period) + 2):
        a.append(2.0 / L * ((sim.moments()[0] - 1) * s).sum())
        sim.step(1)
    zc = [i + a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1) if a[i] * a[i + 1] < 0]
    return period / (2 * np.mean(np.diff(zc)))


@pytest.mark.parametrize("lat", [0, 1])
def test_sound_speed_is_adiabatic(oracle_mod, lat):
    e32 = abs(sound_frequency_ratio(oracle_mod, lat, 32) - 1)
    e64 = abs(sound_frequency_ratio(oracle_mod, lat, 64) - 1)
    assert e64 < 3e-4
    assert 3.0 < e32 / e64 < 5.0  # O(k^2)
