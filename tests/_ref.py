"""Reference closed forms shared by the CPU pin tests (independent of the oracle)."""
import itertools

import numpy as np


def explicit_hermite(xi, n):
    """Closed forms of the tensor Hermite polynomials up to rank 4."""
    D = xi.shape[0]
    d = np.eye(D)
    if n == 0:
        return np.array(1.0)
    if n == 1:
        return xi.copy()
    if n == 2:
        return np.einsum("a,b->ab", xi, xi) - d
    if n == 3:
        t = np.einsum("a,b,c->abc", xi, xi, xi)
        t -= np.einsum("a,bc->abc", xi, d) + np.einsum("b,ac->abc", xi, d) + np.einsum("c,ab->abc", xi, d)
        return t
    if n == 4:
        xx = np.einsum("a,b->ab", xi, xi)
        t = np.einsum("ab,cd->abcd", xx, xx)
        for spec in ("ab,cd", "ac,bd", "ad,bc", "cd,ab", "bd,ac", "bc,ad"):
            t -= np.einsum(spec + "->abcd", xx, d)
        for spec in ("ab,cd", "ac,bd", "ad,bc"):
            t += np.einsum(spec + "->abcd", d, d)
        return t
    raise ValueError(n)


def gh_rule(D, npts=10):
    """Product Gauss-Hermite rule for the unit Gaussian weight in D dimensions:
    nodes (M, D) and weights (M,) summing to one; exact for polynomials of
    degree <= 2*npts - 1 in each variable."""
    x, w = np.polynomial.hermite_e.hermegauss(npts)
    w = w / np.sqrt(2.0 * np.pi)
    nodes = np.array(list(itertools.product(x, repeat=D)))
    weights = np.array([np.prod(t) for t in itertools.product(w, repeat=D)])
    return nodes, weights


def maxwellian_average(D, rho, u, theta, fn, npts=10):
    """Integral of the Maxwellian f0(rho, u, theta) times fn(xi), computed by
    the substitution xi = u + sqrt(theta) eta and a product Gauss-Hermite rule
    (exact when fn is a polynomial of degree < 2*npts)."""
    nodes, weights = gh_rule(D, npts)
    u = np.asarray(u, dtype=np.float64)[:D]
    acc = None
    for eta, wt in zip(nodes, weights):
        val = wt * np.asarray(fn(u + np.sqrt(theta) * eta))
        acc = val if acc is None else acc + val
    return rho * acc


def outer_power(v, k):
    t = np.array(1.0)
    for _ in range(k):
        t = np.multiply.outer(t, v)
    return t
