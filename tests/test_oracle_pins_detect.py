"""The oracle's pins are sharp: a plausible mistake planted in the oracle's
inputs (on the CPU) makes the corresponding pin fail.

Each case recomputes element matrices with a deliberately wrong tabulation
(swapped derivative slabs, a flipped sign, a dropped or misplaced quadrature
weight) and checks that the closed form or exact integral used as a pin in
test_oracle_local.py / test_oracle_global.py is then violated by far more
than that pin's tolerance.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from fe_inputs import config_mesh
from fe_inputs.meshes import nodal_values


def _p1_tet_error(tab_mutator):
    """Largest relative deviation from the P1 tetrahedron closed form."""
    rng = np.random.default_rng(11)
    cells = rng.uniform(0, 1, size=(8, 4, 3))
    pts, w, vals, grads = oracle.tabulation(3, 1, 0)
    tab = tab_mutator((pts, w.copy(), vals.copy(), grads.copy()))
    K = oracle.local_matrices("stiffness", cells, 1, 0, tab=tab)
    worst = 0.0
    for c, x in enumerate(cells):
        Mx = np.hstack([np.ones((4, 1)), x])
        vol = abs(np.linalg.det(Mx)) / 6
        g = np.linalg.inv(Mx)[1:, :].T
        Kc = vol * g @ g.T
        worst = max(worst, np.abs(K[c] - Kc).max() / np.abs(Kc).max())
    return worst


def _identity(tab):
    return tab


def _swap_slabs(tab):
    pts, w, vals, grads = tab
    return pts, w, vals, grads[[1, 0, 2]]          # d/dX and d/dY exchanged


def _flip_sign(tab):
    pts, w, vals, grads = tab
    grads = grads.copy()
    grads[2] *= -1.0
    return pts, w, vals, grads


def test_p1_closed_form_pin_is_sharp():
    assert _p1_tet_error(_identity) < 1e-12
    # a transposed operand or a wrong sign on one derivative is caught
    assert _p1_tet_error(_swap_slabs) > 1e-3
    assert _p1_tet_error(_flip_sign) > 1e-3


def _global(form, m, q, tab):
    A = oracle.local_matrices(form, m.cell_coords, m.degree, q, m.dofmap, tab=tab)
    rp, ci, v = oracle.assemble(m.dofmap, A, m.n_dofs)
    return sp.csr_matrix((v, ci, rp), shape=(m.n_dofs, m.n_dofs))


@pytest.mark.parametrize("mistake", ["none", "drop_weight", "shift_weights"])
def test_exact_mass_integral_pin_is_sharp(mistake):
    m = config_mesh("c2", n=2, flatten=0.0)
    pts, w, vals, grads = oracle.tabulation(3, 4, 8)
    w = w.copy()
    if mistake == "drop_weight":
        w[0] = 0.0                                  # a dropped term of the rule
    elif mistake == "shift_weights":
        w = np.roll(w, 1)                           # weights paired with the wrong points
    M = _global("mass", m, 8, (pts, w, vals, grads))
    u = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] ** 2 * x[:, 1])
    v = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 2] ** 2)
    err = abs(u @ (M @ v) - 1.0 / 18.0)
    if mistake == "none":
        assert err < 1e-14
    else:
        assert err > 1e-6


@pytest.mark.parametrize("mistake", ["none", "swap_slabs", "flip_sign"])
def test_exact_stiffness_integral_pin_is_sharp(mistake):
    m = config_mesh("c2", n=2, flatten=0.0)
    tab = {"none": _identity, "swap_slabs": _swap_slabs, "flip_sign": _flip_sign}[mistake](
        oracle.tabulation(3, 4, 8))
    K = _global("stiffness", m, 8, tab)
    u = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] ** 2 * x[:, 1])
    w = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] * x[:, 1] * x[:, 2])
    err = abs(u @ (K @ w) - 7.0 / 24.0)
    if mistake == "none":
        assert err < 1e-13
    else:
        assert err > 1e-3


def _local_action_sum(form, m, q, tab, u, w):
    b, _ = oracle.local_vectors(form, m.cell_coords, m.degree, q, m.dofmap, u, tab=tab)
    return w @ oracle.assemble_vector(m.dofmap, b, m.n_dofs)


@pytest.mark.parametrize("mistake", ["none", "swap_slabs", "flip_sign"])
def test_action_exact_integral_pin_is_sharp(mistake):
    m = config_mesh("c2", n=2, flatten=0.0)
    tab = {"none": _identity, "swap_slabs": _swap_slabs, "flip_sign": _flip_sign}[mistake](
        oracle.tabulation(3, 4, 8))
    u = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] ** 2 * x[:, 1])
    w = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] * x[:, 1] * x[:, 2])
    err = abs(_local_action_sum("stiffness", m, 8, tab, u, w) - 7.0 / 24.0)
    assert (err < 1e-13) if mistake == "none" else (err > 1e-3)


@pytest.mark.parametrize("mistake", ["none", "drop_weight", "shift_weights"])
def test_mass_action_constant_pin_is_sharp(mistake):
    m = config_mesh("c2", n=2, flatten=0.0)
    pts, w, vals, grads = oracle.tabulation(3, 4, 8)
    w = w.copy()
    if mistake == "drop_weight":
        w[0] = 0.0
    elif mistake == "shift_weights":
        w = np.roll(w, 1)
    one = np.ones(m.n_dofs)
    u = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, lambda x: x[:, 0] ** 4)
    # int x^4 = 1/5 through the mass action; the constant sum alone does not
    # see a permutation of the weights, the degree-4 integrand does
    err = abs(_local_action_sum("mass", m, 8, (pts, w, vals, grads), u, one) - 0.2)
    assert (err < 1e-13) if mistake == "none" else (err > 1e-6)


@pytest.mark.parametrize("mistake", ["none", "swap_slabs", "flip_sign"])
def test_adjoint_exact_integral_pin_is_sharp(mistake):
    m = config_mesh("c2", n=2, flatten=0.0)
    tab = {"none": _identity, "swap_slabs": _swap_slabs, "flip_sign": _flip_sign}[mistake](
        oracle.tabulation(3, 4, 8))
    nv = lambda f: nodal_values(m.cell_coords, m.dofmap, m.n_dofs, 4, f)  # noqa: E731
    u, v, w = nv(lambda x: x[:, 0] ** 2 * x[:, 1]), nv(lambda x: x[:, 0] * x[:, 2]), \
        nv(lambda x: x[:, 0] * x[:, 1])
    _, g = oracle.local_vectors("stiffness", m.cell_coords, 4, 8, m.dofmap, u,
                                coeff=np.ones(m.n_dofs), v=v, tab=tab)
    err = abs(w @ oracle.assemble_vector(m.dofmap, g, m.n_dofs) - 1.0 / 9.0)
    assert (err < 1e-13) if mistake == "none" else (err > 1e-3)
