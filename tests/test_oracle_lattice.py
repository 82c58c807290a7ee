"""Pins of the oracle's quadrature rules and Hermite tensors (CPU only).

* Gauss-Hermite exactness of the derived rules (paper Sec. 2, the degree-Q rule
  that turns eq. (an) into eq. (an1)): exact through degree 9 (D2Q37) and 7
  (D3Q39), inexact one degree higher.
* The D2Q37 lattice constant printed in the paper's Sec. 3 (golden file).
* The D2Q37 and D3Q39 weights against the published E^9_{2,37} and E^7_{3,39}
  rules (golden files).
* Hermite tensors of the oracle against their explicit closed forms and against
  the orthogonality relation they must satisfy under an exact rule.
"""
import itertools
import os

import numpy as np
import pytest

from _ref import explicit_hermite

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gaussian_moment(p):
    """Integral of omega(xi) prod_a xi_a^p_a for the unit Gaussian weight."""
    out = 1.0
    for k in p:
        if k % 2:
            return 0.0
        out *= float(np.prod(np.arange(k - 1, 0, -2))) if k > 0 else 1.0
    return out


def quad_error(xi, w, p):
    m = np.sum(w * np.prod(xi ** np.asarray(p)[None, :], axis=1))
    return abs(m - gaussian_moment(p))


@pytest.mark.parametrize("lat,Q,D,deg", [(0, 37, 2, 9), (1, 39, 3, 7)])
def test_rule_is_gauss_hermite_of_stated_degree(oracle_mod, lat, Q, D, deg):
    c, w, r, degree = oracle_mod.lattice(lat)
    assert len(w) == Q and degree == deg
    xi = r * c[:, :D].astype(np.float64)
    assert np.all(w > 0)
    for tot in range(deg + 1):
        for p in itertools.product(range(tot + 1), repeat=D):
            if sum(p) != tot:
                continue
            assert quad_error(xi, w, p) < 1e-13 * max(1.0, gaussian_moment(p)), p
    worst = max(quad_error(xi, w, p) for p in itertools.product(range(deg + 2), repeat=D)
                if sum(p) == deg + 1)
    assert worst > 1e-3, "rule should not be exact one degree higher"


@pytest.mark.parametrize("lat", [0, 1])
def test_velocity_set_symmetric_and_integer(oracle_mod, lat):
    c, w, r, _ = oracle_mod.lattice(lat)
    vecs = {tuple(v) for v in c}
    assert len(vecs) == len(c)
    for v, wv in zip(c, w):
        assert tuple(-v) in vecs
    assert np.abs(c).max() == 3  # streaming reaches three nodes per axis


def test_d2q37_lattice_constant_matches_paper(oracle_mod):
    with open(os.path.join(GOLDEN, "d2q37_lattice_constant.txt")) as fh:
        printed = float([l for l in fh if not l.startswith("#") and l.strip()][0])
    _, _, r, _ = oracle_mod.lattice(0)
    assert abs(r - printed) < 5e-6  # six significant digits


def test_d3q39_scale_is_sqrt_three_halves(oracle_mod):
    # The degree-7 D3Q39 rule has r^2 = 3/2 and a rest weight of exactly 1/12.
    c, w, r, _ = oracle_mod.lattice(1)
    assert abs(r * r - 1.5) < 1e-15
    rest = w[np.all(c == 0, axis=1)][0]
    assert abs(rest - 1.0 / 12.0) < 1e-16


def test_d3q39_weights_match_the_published_rule(oracle_mod):
    """Every shell weight of the derived D3Q39 rule equals the published
    E^7_{3,39} table (golden file, exact fractions), and so does r^2."""
    from fractions import Fraction

    shells = {}
    r2 = None
    with open(os.path.join(GOLDEN, "d3q39_weights.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if f[0] == "r2":
                r2 = float(Fraction(f[1]))
            else:
                shells[tuple(int(v) for v in f[:3])] = (int(f[3]), float(Fraction(f[4])))
    c, w, r, _ = oracle_mod.lattice(1)
    assert abs(r * r - r2) < 1e-15
    seen = {}
    for v, wv in zip(c, w):
        gen = tuple(sorted((abs(int(a)) for a in v[:3]), reverse=True))
        assert gen in shells, gen
        assert abs(wv - shells[gen][1]) <= 1e-15 * shells[gen][1], (gen, wv)
        seen[gen] = seen.get(gen, 0) + 1
    assert seen == {g: n for g, (n, _) in shells.items()}
    assert abs(sum(n * wt for n, wt in shells.values()) - 1.0) < 1e-15


def test_d2q37_weights_match_the_published_rule(oracle_mod):
    """Every shell weight and the scale r of the derived D2Q37 rule equal the
    23-digit published E^9_{2,37} values (golden file) to FP64 rounding."""
    shells = {}
    r_pub = None
    with open(os.path.join(GOLDEN, "d2q37_weights.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if f[0] == "r":
                r_pub = float(f[1])
            else:
                shells[(int(f[0]), int(f[1]))] = (int(f[2]), float(f[3]))
    c, w, r, _ = oracle_mod.lattice(0)
    assert abs(r - r_pub) <= 4e-16 * r_pub
    seen = {}
    for v, wv in zip(c, w):
        gen = tuple(sorted((abs(int(a)) for a in v[:2]), reverse=True))
        assert gen in shells, gen
        assert abs(wv - shells[gen][1]) <= 1e-15 * shells[gen][1], (gen, wv)
        seen[gen] = seen.get(gen, 0) + 1
    assert seen == {g: n for g, (n, _) in shells.items()}


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
def test_hermite_tensors_closed_form(oracle_mod, lat, n):
    xi = oracle_mod.velocities(lat)
    H = oracle_mod.hermite(lat, n)
    for i in range(len(xi)):
        np.testing.assert_allclose(H[i], explicit_hermite(xi[i], n), rtol=0, atol=1e-13)


def _delta_perm_sum(D, n):
    """sum over permutations pi of prod_k delta(A_k, B_pi(k)), as a rank-2n tensor."""
    out = np.zeros((D,) * (2 * n))
    for idx in itertools.product(range(D), repeat=n):
        for perm in itertools.permutations(range(n)):
            B = tuple(idx[perm[k]] for k in range(n))
            out[idx + B] += 1.0
    return out


@pytest.mark.parametrize("lat,deg", [(0, 9), (1, 7)])
def test_hermite_orthogonality_under_the_rule(oracle_mod, lat, deg):
    _, w, _, _ = oracle_mod.lattice(lat)
    D = 2 if lat == 0 else 3
    for m in range(5):
        for n in range(5):
            if m + n > deg:
                continue
            Hm = oracle_mod.hermite(lat, m).reshape(len(w), -1)
            Hn = oracle_mod.hermite(lat, n).reshape(len(w), -1)
            G = np.einsum("i,ia,ib->ab", w, Hm, Hn)
            if m != n:
                assert np.abs(G).max() < 1e-12, (m, n)
            else:
                ref = _delta_perm_sum(D, n).reshape(D ** n, D ** n)
                np.testing.assert_allclose(G, ref, atol=1e-12)
