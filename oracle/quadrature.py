"""Oracle quadrature: collapsed Gauss-Jacobi rules on the reference simplex (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper assumes a quadrature rule {(w_q, X_q)} that integrates the forms
(Section 3.1, the quadrature footnote allows inexact rules) and takes its
rules from an offline FP64 tabulation (Section 5.1).  The reading used here:
m = floor(q/2) + 1 Gauss-Jacobi points per direction on [0, 1] with weight
(1 - t)^alpha, alpha = 0 for the first collapsed coordinate, 1 for the
second, 2 for the third; the Duffy map
    X = a (1 - b)(1 - c),  Y = b (1 - c),  Z = c      (tetrahedron)
    X = a (1 - b),         Y = b                      (triangle)
with w = w_a w_b (w_c); points ordered with a fastest.  A rule with m points
per direction integrates polynomials of total degree <= 2m - 1 exactly.

The 1D rules come from the Golub-Welsch eigenproblem of the Jacobi matrix
(symmetric tridiagonal), solved with ``numpy.linalg.eigh``.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_jacobi_01(m: int, alpha: int) -> tuple[np.ndarray, np.ndarray]:
    """m-point Gauss rule on [0, 1] for the weight (1 - t)^alpha.

    On [-1, 1] this is Gauss-Jacobi with (a, b) = (alpha, 0); t = (x + 1) / 2.
    Golub-Welsch: nodes are the eigenvalues of the Jacobi matrix built from
    the three-term recurrence of the monic Jacobi polynomials, weights are
    mu_0 times the squared first eigenvector components.
    """
    if m < 1:
        raise ValueError("m >= 1")
    a, b = float(alpha), 0.0
    n = np.arange(m, dtype=np.float64)
    s = 2.0 * n + a + b
    # diagonal: (b^2 - a^2) / (s (s + 2)); n = 0 with a + b = 0 is (b - a)/(a + b + 2)
    diag = np.empty(m)
    for k in range(m):
        den = s[k] * (s[k] + 2.0)
        diag[k] = (b * b - a * a) / den if den != 0.0 else (b - a) / (a + b + 2.0)
    off = np.empty(max(m - 1, 0))
    for k in range(1, m):
        sk = 2.0 * k + a + b
        num = 4.0 * k * (k + a) * (k + b) * (k + a + b)
        den = sk * sk * (sk + 1.0) * (sk - 1.0)
        off[k - 1] = math.sqrt(num / den)
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(T)
    mu0 = 2.0 ** (a + b + 1.0) * math.gamma(a + 1.0) * math.gamma(b + 1.0) / math.gamma(a + b + 2.0)
    w = mu0 * V[0, :] ** 2
    t = 0.5 * (x + 1.0)
    wt = w * 2.0 ** (-(a + b + 1.0))
    return t, wt


def points_per_direction(quad_degree: int) -> int:
    return quad_degree // 2 + 1


def collapsed_rule(d: int, quad_degree: int) -> tuple[np.ndarray, np.ndarray]:
    """Collapsed Gauss-Jacobi rule: (points [n_q][d], weights [n_q])."""
    m = points_per_direction(quad_degree)
    ta, wa = gauss_jacobi_01(m, 0)
    tb, wb = gauss_jacobi_01(m, 1)
    if d == 2:
        A, Bc = np.meshgrid(ta, tb, indexing="xy")          # a fastest
        WA, WB = np.meshgrid(wa, wb, indexing="xy")
        a = A.ravel(); bb = Bc.ravel()
        pts = np.stack([a * (1.0 - bb), bb], axis=1)
        w = (WA * WB).ravel()
        return pts, w
    if d == 3:
        tc, wc = gauss_jacobi_01(m, 2)
        C, Bc, A = np.meshgrid(tc, tb, ta, indexing="ij")  # a fastest, c slowest
        WC, WB, WA = np.meshgrid(wc, wb, wa, indexing="ij")
        a = A.ravel(); bb = Bc.ravel(); c = C.ravel()
        pts = np.stack([a * (1.0 - bb) * (1.0 - c), bb * (1.0 - c), c], axis=1)
        w = (WA * WB * WC).ravel()
        return pts, w
    raise ValueError("d must be 2 or 3")
