"""Pins for the oracle's actions (Algorithm 2) and coefficient adjoint.

The action y = A(z) u is pinned by the Algorithm 1 route (the assembled
matrix, itself pinned in test_oracle_local.py / test_oracle_global.py, times
u), by constants (mass: sum y = |Omega|; stiffness: y = 0) and by exact
polynomial integrals.  The adjoint grad_z[m] = v^T (dA/dz_m) u is pinned by
the exact integral of w grad u . grad v, the Euler identity for a function
linear in z, brute force through the matrix oracle with z = e_m, and central
finite differences of the patch functional.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from fe_inputs import config_mesh, nodal_values
from fe_inputs.meshes import lattice_multi_indices


def _matrix(form, m, q, coeff=None):
    rp, ci, v = oracle.assemble_form(form, m, q, coeff=coeff)
    return sp.csr_matrix((v, ci, rp), shape=(m.n_dofs, m.n_dofs))


def _kappa(x):
    return 1.0 + x[:, 0] * x[:, 1] + 0.5 * x[:, 2] ** 2


@pytest.mark.parametrize("form,p,q,with_coeff", [
    ("mass", 2, 4, False), ("stiffness", 2, 4, False), ("mass", 4, 8, True),
    ("stiffness", 4, 8, False), ("stiffness", 3, 6, True),
])
def test_action_equals_matrix_times_vector(form, p, q, with_coeff):
    m = config_mesh("c2", n=2, degree=p, flatten=0.05)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(m.n_dofs)
    z = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, p, _kappa) if with_coeff else None
    y = oracle.action(form, m, q, u, coeff=z)
    ref = _matrix(form, m, q, z) @ u
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p,q", [(2, 4), (4, 8)])
def test_actions_on_constants(p, q):
    m = config_mesh("c2", n=3, degree=p, flatten=0.0)
    one = np.ones(m.n_dofs)
    y_mass = oracle.action("mass", m, q, one)
    assert abs(y_mass.sum() - 1.0) < 1e-13          # 1^T M 1 = |unit cube|
    y_stiff = oracle.action("stiffness", m, q, one)
    assert np.abs(y_stiff).max() < 1e-12            # constants are in the kernel


def test_action_exact_integral_and_triangles():
    # v^T (A u) = int grad u . grad v for polynomials the space reproduces
    m = config_mesh("c2", n=2, degree=4, flatten=0.0)
    u = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] ** 2 * x[:, 1])
    w = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] * x[:, 1] * x[:, 2])
    assert abs(w @ oracle.action("stiffness", m, 8, u) - 7.0 / 24.0) < 1e-13
    t = config_mesh("c1", n=4, degree=2)
    rng = np.random.default_rng(1)
    ut = rng.standard_normal(t.n_dofs)
    ref = _matrix("stiffness", t, 2) @ ut
    assert np.abs(oracle.action("stiffness", t, 2, ut) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("form,expected", [
    # sum_m g_m w_m = int w grad u . grad v with u = x^2 y, v = x z, w = x y:
    # grad u . grad v = 2xyz, so the integral is 2 (1/3)(1/3)(1/2) = 1/9
    ("stiffness", 1.0 / 9.0),
    # mass: int w u v = int x^4 y^2 z = (1/5)(1/3)(1/2) = 1/30
    ("mass", 1.0 / 30.0),
])
def test_adjoint_exact_integral(form, expected):
    m = config_mesh("c2", n=2, degree=4, flatten=0.0)
    nv = lambda f: nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, f)  # noqa: E731
    u = nv(lambda x: x[:, 0] ** 2 * x[:, 1])
    v = nv(lambda x: x[:, 0] * x[:, 2])
    w = nv(lambda x: x[:, 0] * x[:, 1])
    z = nv(_kappa)                                   # g does not depend on z
    _, g = oracle.vjp(form, m, 8, u, v, coeff=z)
    assert abs(g @ w - expected) < 1e-13


@pytest.mark.parametrize("form", ["mass", "stiffness"])
def test_adjoint_euler_identity_and_grad_u(form):
    m = config_mesh("c2", n=2, degree=3, flatten=0.05)
    rng = np.random.default_rng(2)
    u, v = rng.standard_normal(m.n_dofs), rng.standard_normal(m.n_dofs)
    z = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 3, _kappa)
    gu, gz = oracle.vjp(form, m, 6, u, v, coeff=z)
    A = _matrix(form, m, 6, z)
    f = v @ (A @ u)
    assert abs(z @ gz - f) <= 1e-12 * np.abs(gz).sum() * np.abs(z).max()
    ref = A.T @ v
    assert np.abs(gu - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("form", ["mass", "stiffness"])
def test_adjoint_brute_force_unit_coefficients(form):
    m = config_mesh("c2", n=1, degree=2, flatten=0.0)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(m.n_dofs), rng.standard_normal(m.n_dofs)
    _, gz = oracle.vjp(form, m, 4, u, v, coeff=np.ones(m.n_dofs))
    for k in range(m.n_dofs):
        e = np.zeros(m.n_dofs)
        e[k] = 1.0
        ref = v @ (_matrix(form, m, 4, e) @ u)
        assert abs(gz[k] - ref) <= 1e-12 * max(1.0, abs(ref))


def _dof_kind(m, p):
    """0 vertex, 1 edge, 2 face, 3 interior: nonzero barycentric indices - 1."""
    alpha = lattice_multi_indices(3, p)
    lam = np.concatenate([p - alpha.sum(axis=1, keepdims=True), alpha], axis=1)
    kind_local = (lam > 0).sum(axis=1) - 1
    kind = np.zeros(m.n_dofs, dtype=np.int64)
    kind[m.dofmap.reshape(-1)] = np.tile(kind_local, m.dofmap.shape[0])
    return kind


def test_adjoint_central_differences_patch_functional():
    # f is linear in z, so central differences with h = 1e-6 in FP64 are exact
    # up to rounding; the patch functional (cells containing dof m only) keeps
    # the cancellation small.  64 dofs drawn by seed 3 over all dof kinds.
    p, q = 4, 8
    m = config_mesh("c2", n=2, degree=p, flatten=0.05)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(m.n_dofs), rng.standard_normal(m.n_dofs)
    z = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, p, _kappa)
    _, gz = oracle.vjp("stiffness", m, q, u, v, coeff=z)
    kind = _dof_kind(m, p)
    picks = np.concatenate([rng.choice(np.flatnonzero(kind == k), 16, replace=False)
                            for k in range(4)])
    h = 1e-6
    for dof in picks:
        cells = np.flatnonzero((m.dofmap == dof).any(axis=1))
        A_loc = lambda zz: oracle.local_matrices("stiffness", m.cell_coords[cells], p, q,  # noqa
                                                 m.dofmap[cells], zz)
        zp, zm = z.copy(), z.copy()
        zp[dof] += h
        zm[dof] -= h
        fp = sum(v[m.dofmap[c]] @ A @ u[m.dofmap[c]] for c, A in zip(cells, A_loc(zp)))
        fm = sum(v[m.dofmap[c]] @ A @ u[m.dofmap[c]] for c, A in zip(cells, A_loc(zm)))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - gz[dof]) <= 1e-6 * max(1.0, abs(gz[dof])), (dof, fd, gz[dof])
