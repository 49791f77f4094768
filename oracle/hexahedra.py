"""Oracle for hexahedral (boxed) cells: mass matrices with per-point geometry (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Reference cell: the unit cube [0, 1]^3 (Section 5.1).  Basis: tensor
products of 1D Lagrange polynomials on the equispaced nodes k / p, local
index i + (p+1)(j + (p+1)k) (x fastest).  Quadrature: the tensor product of
the m-point Gauss-Legendre rule on [0, 1], m = floor(q/2) + 1, x fastest.
Geometry: the trilinear map x(X) = sum_v x_v phi_v(X) over the 8 vertices
(vertex v at the reference corner (v & 1, (v >> 1) & 1, (v >> 2) & 1)); on a
boxed cell J and det J vary in space (Section 4.2, the geometry tensor
G(X) = |det J(X)| of the mass form).  The mass matrix is
A = B^T diag_q(w_q |det J(X_q)|) B, B[q][k] = phi_k(X_q) (Algorithm 1 with
n_d = 1 and a per-point C).
"""
from __future__ import annotations

import numpy as np

from .quadrature import gauss_jacobi_01


def tensor_rule(quad_degree: int):
    """(points [m^3][3], weights [m^3]) on [0, 1]^3, x fastest."""
    m = quad_degree // 2 + 1
    t, w = gauss_jacobi_01(m, 0)
    a, b, c = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    a, b, c = a.T.ravel(), b.T.ravel(), c.T.ravel()          # a fastest
    pts = np.stack([t[a], t[b], t[c]], axis=1)
    return pts, w[a] * w[b] * w[c]


def lagrange_1d(p: int, t: np.ndarray):
    """Values [n][p+1] and derivatives [n][p+1] of the equispaced Lagrange
    polynomials L_k(t) = prod_{a != k} (t - a/p) / (k/p - a/p)."""
    t = np.asarray(t, dtype=np.float64)
    nodes = np.arange(p + 1) / p
    val = np.ones((t.size, p + 1))
    der = np.zeros((t.size, p + 1))
    for k in range(p + 1):
        others = [a for a in range(p + 1) if a != k]
        den = np.prod([nodes[k] - nodes[a] for a in others])
        val[:, k] = np.prod([t - nodes[a] for a in others], axis=0) / den if others else 1.0
        # derivative: sum over the factor left out
        for skip in others:
            rest = [t - nodes[a] for a in others if a != skip]
            der[:, k] += (np.prod(rest, axis=0) if rest else 1.0) / den
    return val, der


def tabulate(p: int, X: np.ndarray):
    """(values [n][n_phi], gradients [3][n][n_phi]) of Q_p at the points X [n][3]."""
    n1 = p + 1
    v = [lagrange_1d(p, X[:, e]) for e in range(3)]
    vals = np.einsum("qi,qj,qk->qkji", v[0][0], v[1][0], v[2][0]).reshape(len(X), -1)
    gx = np.einsum("qi,qj,qk->qkji", v[0][1], v[1][0], v[2][0]).reshape(len(X), -1)
    gy = np.einsum("qi,qj,qk->qkji", v[0][0], v[1][1], v[2][0]).reshape(len(X), -1)
    gz = np.einsum("qi,qj,qk->qkji", v[0][0], v[1][0], v[2][1]).reshape(len(X), -1)
    assert vals.shape[1] == n1 ** 3
    return vals, np.stack([gx, gy, gz])


def jacobian(x8: np.ndarray, X: np.ndarray) -> np.ndarray:
    """J(X) [n][3][3] of the trilinear map of vertices x8 [8][3]."""
    J = np.zeros((len(X), 3, 3))
    for v in range(8):
        bits = [(v >> e) & 1 for e in range(3)]
        f = np.stack([X[:, e] if bits[e] else 1.0 - X[:, e] for e in range(3)], axis=1)
        s = np.array([1.0 if b else -1.0 for b in bits])
        grad = np.stack([s[0] * f[:, 1] * f[:, 2], f[:, 0] * s[1] * f[:, 2],
                         f[:, 0] * f[:, 1] * s[2]], axis=1)              # d phi_v / d X_j
        J += x8[v][None, :, None] * grad[:, None, :]
    return J


def mass_matrices(cell_coords: np.ndarray, p: int, quad_degree: int) -> np.ndarray:
    """A_K [n_cells][n_phi][n_phi] of the mass form on trilinear hexahedra."""
    pts, w = tensor_rule(quad_degree)
    B, _ = tabulate(p, pts)
    out = np.empty((len(cell_coords), B.shape[1], B.shape[1]))
    for K, x8 in enumerate(np.asarray(cell_coords, dtype=np.float64)):
        c = w * np.abs(np.linalg.det(jacobian(x8, pts)))
        out[K] = B.T @ (c[:, None] * B)
    return out
