"""Pins for the oracle's collapsed Gauss-Jacobi rules (not the GPU path)."""
from fractions import Fraction
from math import factorial

import mpmath
import numpy as np
import pytest
import scipy.special

from oracle import quadrature


def exact_simplex_monomial(d, exps):
    """int_T X^i Y^j (Z^k) over the reference simplex = prod(e!) / (|e| + d)!."""
    num = 1
    for e in exps:
        num *= factorial(e)
    return Fraction(num, factorial(sum(exps) + d))


@pytest.mark.parametrize("d,q", [(2, 0), (2, 4), (3, 0), (3, 2), (3, 8), (3, 14), (3, 16)])
def test_weight_sum_is_volume(d, q):
    _, w = quadrature.collapsed_rule(d, q)
    assert abs(w.sum() - 1.0 / factorial(d)) < 1e-15


@pytest.mark.parametrize("d,q,npts", [(2, 0, 1), (3, 0, 1), (3, 8, 125), (3, 14, 512), (3, 16, 729)])
def test_point_counts(d, q, npts):
    pts, w = quadrature.collapsed_rule(d, q)
    assert pts.shape == (npts, d) and w.shape == (npts,)
    assert np.all(w > 0)
    # every point strictly inside the reference simplex
    assert np.all(pts > 0) and np.all(pts.sum(axis=1) < 1)


@pytest.mark.parametrize("d,q", [(2, 4), (2, 6), (3, 4), (3, 8)])
def test_exact_on_monomials(d, q):
    """Exact for every monomial of total degree <= 2m - 1, m = q//2 + 1."""
    pts, w = quadrature.collapsed_rule(d, q)
    m = quadrature.points_per_direction(q)
    top = 2 * m - 1
    checked = 0
    for i in range(top + 1):
        for j in range(top + 1 - i):
            ks = [None] if d == 2 else range(top + 1 - i - j)
            for k in ks:
                exps = (i, j) if d == 2 else (i, j, k)
                val = np.sum(w * np.prod(pts ** np.array(exps), axis=1))
                ex = float(exact_simplex_monomial(d, exps))
                assert abs(val - ex) <= 2e-15 * max(ex, 1e-300) * 50, (exps, val, ex)
                checked += 1
    assert checked > 10


def test_degree_too_high_is_not_exact():
    """The rule is not exact one degree beyond 2m - 1 (guards against a rule
    accidentally being a different, stronger one)."""
    pts, w = quadrature.collapsed_rule(3, 2)      # m = 2: exact to degree 3
    val = np.sum(w * pts[:, 2] ** 4)
    ex = float(exact_simplex_monomial(3, (0, 0, 4)))
    assert abs(val - ex) > 1e-6


@pytest.mark.parametrize("m", [1, 2, 5, 8, 9])
@pytest.mark.parametrize("alpha", [0, 1, 2])
def test_1d_factor_matches_scipy(m, alpha):
    t, w = quadrature.gauss_jacobi_01(m, alpha)
    x, wx = scipy.special.roots_jacobi(m, alpha, 0)
    np.testing.assert_allclose(t, 0.5 * (x + 1.0), rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, wx * 2.0 ** (-(alpha + 1)), rtol=1e-13, atol=0)


@pytest.mark.parametrize("m,alpha", [(5, 1), (8, 2), (9, 0)])
def test_1d_nodes_against_50_digit_roots(m, alpha):
    """Nodes are the zeros of P_m^(alpha,0) mapped to [0,1], refined at 50 digits."""
    mpmath.mp.dps = 50

    def jac(x):
        # explicit sum: P_n^(a,b)(x) = sum_s C(n+a, n-s) C(n+b, s) ((x-1)/2)^s ((x+1)/2)^(n-s)
        return mpmath.fsum(mpmath.binomial(m + alpha, m - s) * mpmath.binomial(m, s)
                           * ((x - 1) / 2) ** s * ((x + 1) / 2) ** (m - s) for s in range(m + 1))

    t, _ = quadrature.gauss_jacobi_01(m, alpha)
    for tk in t:
        root = mpmath.findroot(jac, 2 * mpmath.mpf(tk) - 1)
        assert abs(float((root + 1) / 2) - tk) < 1e-15


def test_centroid_rule():
    for d, vol in [(2, 0.5), (3, 1.0 / 6.0)]:
        pts, w = quadrature.collapsed_rule(d, 0)
        np.testing.assert_allclose(pts[0], np.full(d, 1.0 / (d + 1)), atol=1e-15)
        assert abs(w[0] - vol) < 1e-16
