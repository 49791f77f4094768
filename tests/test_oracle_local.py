"""Pins for the oracle's element matrices (Algorithm 1), not the GPU path."""
import numpy as np
import pytest

import oracle
from fe_inputs import config_mesh


def tri_area(x):
    return 0.5 * abs((x[1, 0] - x[0, 0]) * (x[2, 1] - x[0, 1]) - (x[2, 0] - x[0, 0]) * (x[1, 1] - x[0, 1]))


def test_p1_triangle_closed_forms():
    rng = np.random.default_rng(10)
    cells = rng.uniform(0, 1, size=(20, 3, 2))
    K = oracle.local_matrices("stiffness", cells, 1, 0)
    M = oracle.local_matrices("mass", cells, 1, 2)
    for c, x in enumerate(cells):
        area = tri_area(x)
        b = np.array([x[(i + 1) % 3, 1] - x[(i + 2) % 3, 1] for i in range(3)])
        cc = np.array([x[(i + 2) % 3, 0] - x[(i + 1) % 3, 0] for i in range(3)])
        Kc = (np.outer(b, b) + np.outer(cc, cc)) / (4 * area)
        Mc = area * (1 + np.eye(3)) / 12
        np.testing.assert_allclose(K[c], Kc, rtol=0, atol=1e-13 * np.abs(Kc).max())
        np.testing.assert_allclose(M[c], Mc, rtol=0, atol=1e-14 * np.abs(Mc).max())


def test_p1_tetrahedron_closed_forms():
    rng = np.random.default_rng(11)
    cells = rng.uniform(0, 1, size=(20, 4, 3))
    K = oracle.local_matrices("stiffness", cells, 1, 0)
    M = oracle.local_matrices("mass", cells, 1, 2)
    for c, x in enumerate(cells):
        Mx = np.hstack([np.ones((4, 1)), x])
        vol = abs(np.linalg.det(Mx)) / 6
        C = np.linalg.inv(Mx)              # column i = coefficients of lambda_i
        grads = C[1:, :].T                 # [4][3]
        Kc = vol * grads @ grads.T
        Mc = vol * (1 + np.eye(4)) / 20
        # geometry errors grow like kappa(J) u (Section 4.2): scale the tolerance with it
        tol = 1e-15 * np.linalg.cond(Mx) * 8
        np.testing.assert_allclose(K[c], Kc, rtol=0, atol=tol * np.abs(Kc).max())
        np.testing.assert_allclose(M[c], Mc, rtol=0, atol=tol * np.abs(Mc).max())


@pytest.mark.parametrize("p,q", [(2, 4), (4, 8)])
def test_mass_is_detJ_times_reference(p, q):
    m = config_mesh("c2", n=1, degree=p)
    ref = np.vstack([np.zeros(3), np.eye(3)])[None]
    M_ref = oracle.local_matrices("mass", ref, p, q)[0]
    M = oracle.local_matrices("mass", m.cell_coords, p, q)
    for c in range(m.n_cells):
        _, det, _, _ = oracle.geometry(m.cell_coords[c])
        np.testing.assert_allclose(M[c], abs(det) * M_ref, rtol=0, atol=1e-14 * np.abs(M[c]).max())


@pytest.mark.parametrize("p,q,coef", [(2, 4, False), (4, 8, False), (3, 6, True)])
def test_stiffness_reference_tensor_route(p, q, coef):
    """A_K = sum_st G_st B_s^T diag(w z) B_t computed with dense matrix products."""
    m = config_mesh("c2", n=1, degree=p)
    coeff = None
    if coef:
        coeff = np.random.default_rng(12).uniform(0.5, 2.0, size=m.n_dofs)
    K = oracle.local_matrices("stiffness", m.cell_coords, p, q, m.dofmap, coeff)
    _, w, vals, grads = oracle.tabulation(3, p, q)
    for c in range(m.n_cells):
        _, _, _, G = oracle.geometry(m.cell_coords[c])
        z = np.ones(len(w)) if coeff is None else vals @ coeff[m.dofmap[c]]
        W = np.diag(w * z)
        ref = sum(G[s, t] * grads[s].T @ W @ grads[t] for s in range(3) for t in range(3))
        np.testing.assert_allclose(K[c], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("p,q", [(1, 0), (4, 8), (6, 14)])
def test_symmetry_rowsums_and_volume(p, q):
    m = config_mesh("c2", n=1, degree=p)
    K = oracle.local_matrices("stiffness", m.cell_coords, p, q)
    M = oracle.local_matrices("mass", m.cell_coords, p, max(q, 2 * p))
    for c in range(m.n_cells):
        _, det, _, _ = oracle.geometry(m.cell_coords[c])
        s = np.abs(K[c]).max()
        np.testing.assert_allclose(K[c], K[c].T, atol=1e-14 * s)
        np.testing.assert_allclose(K[c].sum(axis=1), 0.0, atol=1e-12 * s)
        np.testing.assert_allclose(M[c].sum(), abs(det) / 6, rtol=1e-13)


def test_flattened_cells_stay_symmetric_with_large_entries():
    m = config_mesh("c2", n=2, degree=2, flatten=0.2)
    K = oracle.local_matrices("stiffness", m.cell_coords[m.flattened], 2, 4)
    assert np.abs(K).max() > 50.0           # aspect 1e3 inflates gradients
    for Kc in K:
        np.testing.assert_allclose(Kc, Kc.T, atol=1e-13 * np.abs(Kc).max())
        np.testing.assert_allclose(Kc.sum(axis=1), 0.0, atol=1e-11 * np.abs(Kc).max())
