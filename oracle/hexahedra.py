"""Oracle for hexahedral (boxed) cells: mass and Poisson matrices with per-point geometry (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Reference cell: the unit cube [0, 1]^3 (Section 5.1).  Basis: tensor
products of 1D Lagrange polynomials on the equispaced nodes k / p, local
index i + (p+1)(j + (p+1)k) (x fastest).  Quadrature: the tensor product of
the m-point Gauss-Legendre rule on [0, 1], m = floor(q/2) + 1, x fastest.
Geometry: the trilinear map x(X) = sum_v x_v phi_v(X) over the 8 vertices
(vertex v at the reference corner (v & 1, (v >> 1) & 1, (v >> 2) & 1)); on a
boxed cell J and det J vary in space (Section 4.2), so the geometry tensor
G(X) = |det J(X)| (mass) or |det J| J^{-1} J^{-T} (Poisson) is taken at every
quadrature point.  The matrices are Algorithm 1 with a per-point C,
A = sum_s sum_t B_s^T diag_q(w_q G_st(X_q)) B_t; that arithmetic (LU
geometry per point, the triple product) is in the oracle's C part, this
module supplies the rule and the basis tables.
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


def local_matrices(form: str, cell_coords: np.ndarray, p: int, quad_degree: int,
                   nthreads: int = 0) -> np.ndarray:
    """A_K [n_cells][n_phi][n_phi] of the mass or Poisson form on trilinear
    hexahedra: the rule and basis tabulated here, geometry and Algorithm 1
    (with G evaluated at every quadrature point) in the oracle's C part."""
    from . import FORMS, OracleError, _load, _ptr
    pts, w = tensor_rule(quad_degree)
    B, dB = tabulate(p, pts)
    cc = np.ascontiguousarray(cell_coords, dtype=np.float64).reshape(-1, 8, 3)
    pts = np.ascontiguousarray(pts); w = np.ascontiguousarray(w)
    B = np.ascontiguousarray(B); dB = np.ascontiguousarray(dB)
    n_q, n_phi = B.shape
    A = np.empty((len(cc), n_phi, n_phi))
    st = _load().oracle_hex_local_matrices(FORMS[form], len(cc), _ptr(cc), n_phi, n_q, _ptr(pts),
                                           _ptr(w), _ptr(B), _ptr(dB), _ptr(A), int(nthreads))
    if st != 0:
        raise OracleError(f"oracle_hex_local_matrices failed (status {st})")
    return A


def mass_matrices(cell_coords: np.ndarray, p: int, quad_degree: int, nthreads: int = 0) -> np.ndarray:
    """A_K of the mass form on trilinear hexahedra."""
    return local_matrices("mass", cell_coords, p, quad_degree, nthreads)


def stiffness_matrices(cell_coords: np.ndarray, p: int, quad_degree: int,
                       nthreads: int = 0) -> np.ndarray:
    """A_K of the Poisson form on trilinear hexahedra."""
    return local_matrices("stiffness", cell_coords, p, quad_degree, nthreads)
