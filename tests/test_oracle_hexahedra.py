"""Pins for the oracle's hexahedral mass matrices (boxed cells, trilinear
geometry evaluated per quadrature point), independent of the GPU library."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.hexahedra as H
from fe_inputs import hex_mesh


@pytest.mark.parametrize("q", [0, 3, 6, 9])
def test_tensor_rule_integrates_monomials(q):
    pts, w = H.tensor_rule(q)
    m = q // 2 + 1
    for a, b, c in [(2 * m - 1, 0, 0), (1, 2 * m - 1, min(2, 2 * m - 1)), (m, m - 1, 2 * m - 1)]:
        exact = Fraction(1, (a + 1) * (b + 1) * (c + 1))
        got = (w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c).sum()
        assert abs(got - float(exact)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 4])
def test_basis_kronecker_unity_linear(p):
    n1 = p + 1
    idx = np.arange(n1 ** 3)
    nodes = np.stack([idx % n1, (idx // n1) % n1, idx // n1 ** 2], axis=1) / p
    vals, grads = H.tabulate(p, nodes)
    assert np.abs(vals - np.eye(n1 ** 3)).max() < 1e-12           # Kronecker at the lattice
    X = np.random.default_rng(0).uniform(0, 1, (20, 3))
    vals, grads = H.tabulate(p, X)
    assert np.abs(vals.sum(1) - 1).max() < 1e-12
    assert np.abs(grads.sum(2)).max() < 1e-10
    for e in range(3):                                            # linear reproduction
        assert np.abs(vals @ nodes[:, e] - X[:, e]).max() < 1e-12
        assert np.abs(grads[e] @ nodes[:, e] - 1).max() < 1e-10


def _exact_1d_mass(p):
    """int_0^1 L_i L_j with exact rational polynomial arithmetic."""
    nodes = [Fraction(k, p) for k in range(p + 1)]

    def poly(k):                       # coefficients, lowest first
        c = [Fraction(1)]
        for a, xa in enumerate(nodes):
            if a == k:
                continue
            den = nodes[k] - xa
            c = [(c[i - 1] if i else 0) - xa * (c[i] if i < len(c) else 0) for i in range(len(c) + 1)]
            c = [ci / den for ci in c]
        return c
    P = [poly(k) for k in range(p + 1)]
    M = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            prod = [Fraction(0)] * (len(P[i]) + len(P[j]) - 1)
            for a, ca in enumerate(P[i]):
                for b, cb in enumerate(P[j]):
                    prod[a + b] += ca * cb
            M[i, j] = float(sum(c / (n + 1) for n, c in enumerate(prod)))
    return M


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_unit_cube_mass_is_tensor_product_of_exact_1d_mass(p):
    corners = np.array([[(v >> e) & 1 for e in range(3)] for v in range(8)], dtype=float)
    A = H.mass_matrices(corners[None], p, 2 * p)[0]
    M1 = _exact_1d_mass(p)
    ref = np.kron(M1, np.kron(M1, M1))         # index i + (p+1)(j + (p+1)k)
    assert np.abs(A - ref).max() < 1e-14 * np.abs(ref).max() * 10


@pytest.mark.parametrize("p", [1, 3])
def test_jittered_mesh_volume(p):
    m = hex_mesh(3, p, jitter=0.25, seed=4)
    A = H.mass_matrices(m.cell_coords, p, 2 * p)
    assert abs(A.sum() - 1.0) < 1e-13          # the cells tile the unit cube
    assert np.abs(A - A.transpose(0, 2, 1)).max() < 1e-16


def test_uniform_mesh_polynomial_integral():
    # u = x^2 y, v = y z lie in Q_2; the 3-point rule is exact for their product
    m = hex_mesh(2, 2, jitter=0.0)
    A = H.mass_matrices(m.cell_coords, 2, 4)
    rp, ci, vals = oracle.assemble(m.dofmap, A, m.n_dofs)
    M = sp.csr_matrix((vals, ci, rp), shape=(m.n_dofs, m.n_dofs))
    nodes_fn = lambda f: _hex_nodal(m, 2, f)           # noqa: E731
    u = nodes_fn(lambda x: x[:, 0] ** 2 * x[:, 1])
    v = nodes_fn(lambda x: x[:, 1] * x[:, 2])
    assert abs(u @ (M @ v) - 1.0 / 18.0) < 1e-14


def _hex_nodal(m, p, f):
    """Values of f at the nodes of the (unjittered) lattice, by global dof."""
    N = p * m.n + 1
    idx = np.arange(m.n_dofs)
    X = np.stack([idx % N, (idx // N) % N, idx // N ** 2], axis=1) / (N - 1)
    return f(X)


@pytest.mark.parametrize("mistake", ["none", "drop_weight", "local_order"])
def test_pins_are_sharp(mistake, monkeypatch):
    m = hex_mesh(2, 2, jitter=0.0)
    rule = H.tensor_rule
    tab = H.tabulate
    if mistake == "drop_weight":
        def bad_rule(q):
            pts, w = rule(q)
            w = w.copy()
            w[0] = 0.0
            return pts, w
        monkeypatch.setattr(H, "tensor_rule", bad_rule)
    elif mistake == "local_order":
        # local index k + (p+1)(j + (p+1)i) instead of i + (p+1)(j + (p+1)k)
        def bad_tab(p, X):
            v, g = tab(p, X)
            n1 = p + 1
            perm = np.arange(n1 ** 3).reshape(n1, n1, n1).transpose(2, 1, 0).ravel()
            return v[:, perm], g[:, :, perm]
        monkeypatch.setattr(H, "tabulate", bad_tab)
    A = H.mass_matrices(m.cell_coords, 2, 4)
    rp, ci, vals = oracle.assemble(m.dofmap, A, m.n_dofs)
    M = sp.csr_matrix((vals, ci, rp), shape=(m.n_dofs, m.n_dofs))
    u = _hex_nodal(m, 2, lambda x: x[:, 0] ** 2 * x[:, 1])
    v = _hex_nodal(m, 2, lambda x: x[:, 1] * x[:, 2])
    err = abs(u @ (M @ v) - 1.0 / 18.0)
    # a reflected local numbering keeps every integral over a cube (the
    # reflection maps the cell onto itself): the Kronecker pin catches it
    n1 = 3
    idx = np.arange(n1 ** 3)
    nodes = np.stack([idx % n1, (idx // n1) % n1, idx // n1 ** 2], axis=1) / 2
    kron = np.abs(H.tabulate(2, nodes)[0] - np.eye(n1 ** 3)).max()
    if mistake == "none":
        assert err < 1e-14 and kron < 1e-12
    elif mistake == "drop_weight":
        assert err > 1e-4
    else:
        assert kron > 0.5
