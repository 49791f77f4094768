"""Oracle basis: degree-p Lagrange basis on the principal lattice of a simplex (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Appendix A writes simplex Lagrange basis functions as a known constant times a
product of first-degree factors (the Lemma on product-form evaluation, after
Nicolaides), and differentiates such products with the product rule (the
Lemma on derivatives of product-form polynomials).  For equispaced lattice
nodes X_alpha = alpha / p that product is Silvester's:

    phi_alpha(X) = prod_{i=0..d} prod_{j=0..alpha_i-1} (p lambda_i(X) - j) / (j + 1)

with barycentric lambda_0 = 1 - sum_k X_k, lambda_i = X_i, alpha_0 = p - |alpha|.
Local order: alpha_d outermost, alpha_1 innermost.
"""
from __future__ import annotations

import numpy as np


def multi_indices(d: int, p: int) -> np.ndarray:
    out = []
    if d == 2:
        for a2 in range(p + 1):
            for a1 in range(p + 1 - a2):
                out.append((a1, a2))
    elif d == 3:
        for a3 in range(p + 1):
            for a2 in range(p + 1 - a3):
                for a1 in range(p + 1 - a3 - a2):
                    out.append((a1, a2, a3))
    else:
        raise ValueError("d must be 2 or 3")
    return np.asarray(out, dtype=np.int64).reshape(-1, d)


def tabulate(d: int, p: int, X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Values [n_pts][n_phi] and gradients [d][n_pts][n_phi] at points X [n_pts][d]."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, d)
    npts = X.shape[0]
    alphas = multi_indices(d, p)
    nphi = alphas.shape[0]
    lam = np.concatenate([1.0 - X.sum(axis=1, keepdims=True), X], axis=1)   # [n][d+1]
    dlam = np.zeros((d + 1, d))
    dlam[0, :] = -1.0
    for i in range(d):
        dlam[i + 1, i] = 1.0
    vals = np.empty((npts, nphi))
    grads = np.empty((d, npts, nphi))
    for a_idx, a in enumerate(alphas):
        full = np.concatenate([[p - a.sum()], a])
        factors = []       # value arrays [n]
        dfactors = []      # gradient [d] of each factor (constant)
        for i in range(d + 1):
            for j in range(int(full[i])):
                factors.append((p * lam[:, i] - j) / (j + 1))
                dfactors.append(p * dlam[i] / (j + 1))
        v = np.ones(npts)
        for f in factors:
            v = v * f
        vals[:, a_idx] = v
        g = np.zeros((d, npts))
        for k, df in enumerate(dfactors):
            others = np.ones(npts)
            for m, f in enumerate(factors):
                if m != k:
                    others = others * f
            g += df[:, None] * others[None, :]
        grads[:, :, a_idx] = g
    return vals, grads


def n_phi(d: int, p: int) -> int:
    """Dimension of the degree-p simplex Lagrange space: prod_{j=1..d}(p+j)/d!."""
    num = 1
    for j in range(1, d + 1):
        num *= p + j
    den = 1
    for j in range(1, d + 1):
        den *= j
    return num // den
