"""Pins for the oracle's global assembly (Section 3.3), not the GPU path."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from fe_inputs import config_mesh, nodal_values


def dense_brute_force(dofmap, A_local, n_dofs):
    """A^g = sum_K L_K A_K L_K^T with an explicit dense matrix, plus the
    contribution mask (pattern including explicit zeros)."""
    D = np.zeros((n_dofs, n_dofs))
    mask = np.zeros((n_dofs, n_dofs), dtype=bool)
    for K in range(dofmap.shape[0]):
        idx = dofmap[K]
        D[np.ix_(idx, idx)] += A_local[K]
        mask[np.ix_(idx, idx)] = True
    return D, mask


@pytest.mark.parametrize("name,n,p,q,form", [
    ("c1", 1, 1, 0, "stiffness"),
    ("c2", 1, 2, 4, "stiffness"),
    ("c2", 1, 4, 8, "mass"),
    ("c2", 2, 2, 4, "stiffness"),
])
def test_brute_force_dense_assembly(name, n, p, q, form):
    m = config_mesh(name, n=n, degree=p, flatten=0.0)
    A = oracle.local_matrices(form, m.cell_coords, p, q)
    row_ptr, col, vals = oracle.assemble(m.dofmap, A, m.n_dofs)
    D, mask = dense_brute_force(m.dofmap, A, m.n_dofs)
    S = sp.csr_matrix((vals, col, row_ptr), shape=(m.n_dofs, m.n_dofs))
    pattern = sp.csr_matrix((np.ones_like(vals), col, row_ptr), shape=S.shape).toarray() > 0
    np.testing.assert_array_equal(pattern, mask)
    assert row_ptr[-1] == mask.sum()
    for r in range(m.n_dofs):
        assert np.all(np.diff(col[row_ptr[r]:row_ptr[r + 1]]) > 0)
    np.testing.assert_allclose(S.toarray(), D, rtol=0, atol=1e-14 * np.abs(D).max())


def test_counts_c1():
    m = config_mesh("c1")
    row_ptr, col = oracle.csr_pattern(m.dofmap, m.n_dofs)
    assert m.n_dofs == 33 ** 2
    assert row_ptr[-1] == 7361
    pairs = {(int(a), int(b)) for cell in m.dofmap for a in cell for b in cell}
    assert len(pairs) == 7361


@pytest.mark.parametrize("n,p", [(2, 4), (3, 2)])
def test_counts_3d_brute_force(n, p):
    m = config_mesh("c2", n=n, degree=p, flatten=0.0)
    assert m.n_dofs == (p * n + 1) ** 3
    row_ptr, _ = oracle.csr_pattern(m.dofmap, m.n_dofs)
    pairs = {(int(a), int(b)) for cell in m.dofmap for a in cell for b in cell}
    assert row_ptr[-1] == len(pairs)


def test_c1_matches_independent_p1_assembly():
    m = config_mesh("c1")
    row_ptr, col, vals = oracle.assemble_form("stiffness", m, 0)
    rows, cols, data = [], [], []
    for K in range(m.n_cells):
        x = m.cell_coords[K]
        area = 0.5 * abs((x[1, 0] - x[0, 0]) * (x[2, 1] - x[0, 1]) - (x[2, 0] - x[0, 0]) * (x[1, 1] - x[0, 1]))
        b = np.array([x[(i + 1) % 3, 1] - x[(i + 2) % 3, 1] for i in range(3)])
        c = np.array([x[(i + 2) % 3, 0] - x[(i + 1) % 3, 0] for i in range(3)])
        Kc = (np.outer(b, b) + np.outer(c, c)) / (4 * area)
        for i in range(3):
            for j in range(3):
                rows.append(m.dofmap[K, i]); cols.append(m.dofmap[K, j]); data.append(Kc[i, j])
    ref = sp.coo_matrix((data, (rows, cols)), shape=(m.n_dofs, m.n_dofs)).toarray()
    S = sp.csr_matrix((vals, col, row_ptr), shape=ref.shape).toarray()
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def _global(form, m, q, coeff=None):
    rp, ci, v = oracle.assemble_form(form, m, q, coeff=coeff)
    return sp.csr_matrix((v, ci, rp), shape=(m.n_dofs, m.n_dofs))


def test_exact_polynomial_integrals_p4():
    """u^T M v = int u v and u^T K v = int grad u . grad v on the jittered cube."""
    m = config_mesh("c2", n=3, flatten=0.0)          # P4, q = 8, jitter 0.25
    M = _global("mass", m, 8)
    K = _global("stiffness", m, 8)
    u = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] ** 2 * x[:, 1])
    v = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 2] ** 2)
    w = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] * x[:, 1] * x[:, 2])
    one = np.ones(m.n_dofs)
    assert abs(u @ (M @ v) - 1.0 / 18.0) < 1e-14
    assert abs(u @ (K @ w) - 7.0 / 24.0) < 1e-13
    assert abs(one @ (M @ one) - 1.0) < 1e-14
    xs = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0])
    # a sum of nnz(K) ~ 1.4e5 rounded terms of size <= |K|_max: allow nnz * u * |K|_max
    tol = K.nnz * 2.2e-16 * abs(K).max()
    assert abs(xs @ (K @ xs) - 1.0) < tol
    assert np.abs(K @ one).max() < 1e-12 * abs(K).max()


def test_weighted_stiffness_exact_integral_p6():
    """x^T K(kappa) x = int kappa for a degree-6 kappa with q = 14."""
    m = config_mesh("c3", n=2)
    kap = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 6,
                       lambda x: (x[:, 0] * x[:, 1] * x[:, 2]) ** 2)
    K = _global("stiffness", m, 14, coeff=kap)
    xs = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 6, lambda x: x[:, 0])
    assert abs(xs @ (K @ xs) - 1.0 / 27.0) < K.nnz * 2.2e-16 * abs(K).max()


def test_flattened_mesh_mass_sum_is_total_cell_volume():
    m = config_mesh("c2", n=2, degree=2)
    M = _global("mass", m, 4)
    vol = sum(abs(oracle.geometry(x)[1]) / 6 for x in m.cell_coords)
    assert len(m.flattened) > 0
    assert abs(M.sum() - vol) < 1e-14
    assert abs(vol - 1.0) > 1e-3
