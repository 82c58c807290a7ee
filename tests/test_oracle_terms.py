"""Pins of the oracle's per-cell terms: equilibrium and body force (CPU only).

* Maxwellian Hermite coefficients a_0^(n) against a direct quadrature of their
  definition, the integral of f0 H^(n) (paper Sec. 2, eqs. (an) and (f2)).
* Discrete equilibrium moments equal Maxwellian moments up to the expansion
  order (Sec. 2, eqs. (fN), (an1), (rut1)); the truncation shows one order up.
* Discrete force moments (Sec. 2, eq. (F)): zero mass, momentum rho g, second
  moment rho(gu + ug), third Hermite moment from g a^(2) with
  a^(2) = a_0^(2) - sigma (eqs. (f2), (f3)), no heat production (eq. (F-heat)).
* The tensor-built force equals the paper's printed closed form eq. (fi).
* The second-order truncation equals Guo's forcing (the special case stated
  after the mid-point stress in Sec. 2).
"""
import numpy as np
import pytest

from _ref import explicit_hermite, maxwellian_average, outer_power

CASES = [
    (1.0, [0.0, 0.0, 0.0], 1.0),
    (1.3, [0.12, -0.07, 0.05], 1.15),
    (0.8, [-0.2, 0.1, -0.15], 0.85),
]


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("rho,u,theta", CASES)
def test_maxwell_coefficients_by_quadrature(oracle_mod, D, n, rho, u, theta):
    got = oracle_mod.maxwell_coeff(D, n, rho, u[:D], theta)
    ref = maxwellian_average(D, rho, u, theta, lambda xi: explicit_hermite(xi, n), npts=6)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def discrete_moment(xi, f, k):
    return sum(fi * outer_power(x, k) for fi, x in zip(f, xi))


@pytest.mark.parametrize("lat,N", [(0, 4), (0, 3), (0, 2), (1, 3), (1, 2)])
@pytest.mark.parametrize("rho,u,theta", CASES)
def test_equilibrium_moments_equal_maxwellian(oracle_mod, lat, N, rho, u, theta):
    D = 2 if lat == 0 else 3
    xi = oracle_mod.velocities(lat)
    feq = oracle_mod.equilibrium(lat, rho, u[:D], theta, eq_order=N)
    for k in range(N + 1):
        got = discrete_moment(xi, feq, k)
        ref = maxwellian_average(D, rho, u, theta, lambda v: outer_power(v, k), npts=6)
        np.testing.assert_allclose(got, ref, rtol=0, atol=2e-14 * max(1.0, np.abs(ref).max()))
    if any(abs(x) > 0 for x in u) or theta != 1.0:
        # one order above the truncation the moments must differ
        k = N + 1
        got = discrete_moment(xi, feq, k)
        ref = maxwellian_average(D, rho, u, theta, lambda v: outer_power(v, k), npts=6)
        assert np.abs(got - ref).max() > 1e-6


@pytest.mark.parametrize("lat", [0, 1])
def test_equilibrium_default_order(oracle_mod, lat):
    # eq_order 0 selects the highest order the rule supports: 4 (D2Q37), 3 (D3Q39)
    u = [0.1, -0.05, 0.02]
    D = 2 if lat == 0 else 3
    a = oracle_mod.equilibrium(lat, 1.1, u[:D], 1.05, eq_order=0)
    b = oracle_mod.equilibrium(lat, 1.1, u[:D], 1.05, eq_order=4 if lat == 0 else 3)
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        oracle_mod.equilibrium(lat, 1.1, u[:D], 1.05, eq_order=5 if lat == 0 else 4)


def sym3_g_a2(g, a2):
    return (np.einsum("a,bc->abc", g, a2) + np.einsum("b,ac->abc", g, a2)
            + np.einsum("c,ab->abc", g, a2))


FORCE_CASES = [
    (1.0, [0.0, 0.0, 0.0], 1.0, [1e-3, 0.0, 0.0]),
    (1.2, [0.1, -0.05, 0.08], 1.2, [2e-3, -1e-3, 5e-4]),
    (0.9, [-0.15, 0.2, 0.05], 0.8, [-1e-3, 3e-3, 2e-3]),
]


def traceless_sigma(D, seed):
    rng = np.random.default_rng(seed)
    s = rng.normal(size=(D, D)) * 1e-3
    s = 0.5 * (s + s.T)
    return s - np.trace(s) / D * np.eye(D)


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("rho,u,theta,g", FORCE_CASES)
def test_force_hermite_moments(oracle_mod, lat, order, rho, u, theta, g):
    D = 2 if lat == 0 else 3
    u, g = np.asarray(u[:D]), np.asarray(g[:D])
    sig = traceless_sigma(D, 7)
    xi = oracle_mod.velocities(lat)
    F = oracle_mod.force(lat, order, rho, u, theta, g, sig)
    tol = 1e-16
    assert abs(F.sum()) < tol
    np.testing.assert_allclose(discrete_moment(xi, F, 1), rho * g, rtol=0, atol=tol)
    m2 = discrete_moment(xi, F, 2)
    H3 = sum(Fi * explicit_hermite(x, 3) for Fi, x in zip(F, xi))
    heat = sum(Fi * np.dot(x - u, x - u) for Fi, x in zip(F, xi))
    if order == 1:
        np.testing.assert_allclose(m2, 0.0, atol=tol)
        # the first-order term alone produces heat: sum F |xi-u|^2 = -2 rho g.u
        assert abs(heat + 2 * rho * np.dot(g, u)) < tol
        return
    np.testing.assert_allclose(m2, rho * (np.outer(g, u) + np.outer(u, g)), rtol=0, atol=tol)
    assert abs(heat) < tol  # eq. (F-heat): no heat production
    if order == 2:
        np.testing.assert_allclose(H3, 0.0, atol=tol)
        return
    a2 = rho * (np.outer(u, u) + (theta - 1.0) * np.eye(D))
    if order == 4:
        a2 = a2 - sig
    np.testing.assert_allclose(H3, sym3_g_a2(g, a2), rtol=0, atol=tol)


def force_printed(w, xi, rho, u, theta, g, sigma, D):
    """The paper's closed form of the discrete force up to the third moment (eq. (fi))."""
    out = np.empty(len(w))
    for i, (wi, x) in enumerate(zip(w, xi)):
        gx, ux, gu, uu, x2 = g @ x, u @ x, g @ u, u @ u, x @ x
        out[i] = (wi * rho * gx * (1 + ux + 0.5 * (ux * ux - uu + (theta - 1) * (x2 - D - 2)))
                  - wi * rho * gu * (1 + ux)
                  - 0.5 * wi * (gx * (x @ sigma @ x) - 2 * (g @ sigma @ x)))
    return out


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("rho,u,theta,g", FORCE_CASES)
def test_force_matches_printed_closed_form(oracle_mod, lat, rho, u, theta, g):
    D = 2 if lat == 0 else 3
    u, g = np.asarray(u[:D]), np.asarray(g[:D])
    sig = traceless_sigma(D, 11)
    _, w, _, _ = oracle_mod.lattice(lat)
    xi = oracle_mod.velocities(lat)
    F = oracle_mod.force(lat, 4, rho, u, theta, g, sig)
    np.testing.assert_allclose(F, force_printed(w, xi, rho, u, theta, g, sig, D),
                               rtol=0, atol=1e-17)
    # without sigma (force order 3) the printed form with sigma = 0
    F3 = oracle_mod.force(lat, 3, rho, u, theta, g, sig)
    np.testing.assert_allclose(F3, force_printed(w, xi, rho, u, theta, g, 0 * sig, D),
                               rtol=0, atol=1e-17)


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("rho,u,theta,g", FORCE_CASES)
def test_second_order_truncation_is_guo_forcing(oracle_mod, lat, rho, u, theta, g):
    D = 2 if lat == 0 else 3
    u, g = np.asarray(u[:D]), np.asarray(g[:D])
    _, w, _, _ = oracle_mod.lattice(lat)
    xi = oracle_mod.velocities(lat)
    F2 = oracle_mod.force(lat, 2, rho, u, theta, g)
    # Guo, Zheng & Shi (2002) source with unit reference temperature (c_s^2 = 1):
    # w_i rho [(xi_i - u).g + (xi_i.u)(xi_i.g)]
    guo = np.array([wi * rho * ((x - u) @ g + (x @ u) * (x @ g)) for wi, x in zip(w, xi)])
    np.testing.assert_allclose(F2, guo, rtol=0, atol=1e-17)
    F1 = oracle_mod.force(lat, 1, rho, u, theta, g)
    np.testing.assert_allclose(F1, w * rho * (xi @ g), rtol=0, atol=1e-17)
    # the first two moments agree for every order >= 2
    for order in (3, 4):
        Fo = oracle_mod.force(lat, order, rho, u, theta, g, traceless_sigma(D, 3))
        for k in (0, 1, 2):
            np.testing.assert_allclose(discrete_moment(xi, Fo, k), discrete_moment(xi, F2, k),
                                       rtol=0, atol=1e-16)
