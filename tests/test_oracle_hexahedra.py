"""Pins for the oracle's hexahedral mass and Poisson matrices (boxed cells,
trilinear geometry evaluated per quadrature point), independent of the GPU
library."""
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


def _exact_1d_mass(p, deriv=False):
    """int_0^1 L_i L_j (or L_i' L_j' with deriv) with exact rational
    polynomial arithmetic."""
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
    if deriv:
        P = [[n * c for n, c in enumerate(pk)][1:] or [Fraction(0)] for pk in P]
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

@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_unit_cube_stiffness_is_kronecker_sum_of_exact_1d_matrices(p):
    corners = np.array([[(v >> e) & 1 for e in range(3)] for v in range(8)], dtype=float)
    A = H.stiffness_matrices(corners[None], p, 2 * p)[0]
    M1, K1 = _exact_1d_mass(p), _exact_1d_mass(p, deriv=True)
    # index i + (p+1)(j + (p+1)k): the last Kronecker factor is x
    ref = (np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1)) +
           np.kron(K1, np.kron(M1, M1)))
    assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()


def _hex_node_positions(m, p):
    """Physical position of every global dof: the trilinear map of its cell
    at the reference lattice point (shared nodes get one position: the map
    on a face depends only on the face's vertices)."""
    n1 = p + 1
    idx = np.arange(n1 ** 3)
    X = np.stack([idx % n1, (idx // n1) % n1, idx // n1 ** 2], axis=1) / p
    phi = np.ones((len(X), 8))
    for v in range(8):
        for e in range(3):
            phi[:, v] *= X[:, e] if (v >> e) & 1 else 1.0 - X[:, e]
    pos = np.zeros((m.n_dofs, 3))
    for K in range(m.cell_coords.shape[0]):
        pos[m.dofmap[K]] = phi @ m.cell_coords[K]
    return pos


def _stiffness_pins(m, p, q):
    """(max |K 1| / max|K|, max_e |x_e^T K x_e - 1|, symmetry defect)."""
    A = H.stiffness_matrices(m.cell_coords, p, q)
    rp, ci, vals = oracle.assemble(m.dofmap, A, m.n_dofs)
    K = sp.csr_matrix((vals, ci, rp), shape=(m.n_dofs, m.n_dofs))
    pos = _hex_node_positions(m, p)
    rows = np.abs(K @ np.ones(m.n_dofs)).max() / np.abs(vals).max()
    energy = max(abs(pos[:, e] @ (K @ pos[:, e]) - 1.0) for e in range(3))
    sym = np.abs(A - A.transpose(0, 2, 1)).max() / np.abs(A).max()
    return rows, energy, sym


@pytest.mark.parametrize("p", [1, 2, 3])
def test_jittered_mesh_stiffness_rows_and_coordinate_energy(p):
    # the coordinate functions lie in Q_1 on every trilinear cell, so
    # x^T K x = int |grad x|^2 = |Omega| = 1; |det J| has degree <= 2 per
    # variable, integrated exactly by m >= 2 points per direction
    m = hex_mesh(3, p, jitter=0.25, seed=4)
    rows, energy, sym = _stiffness_pins(m, p, 2 * p)
    assert rows < 1e-13 and energy < 1e-13 and sym < 1e-15, (rows, energy, sym)


def test_uniform_mesh_stiffness_polynomial_integral():
    # u = x^2 y, v = y z in Q_2: int grad u . grad v = int x^2 z = 1/6
    m = hex_mesh(2, 2, jitter=0.0)
    A = H.stiffness_matrices(m.cell_coords, 2, 4)
    rp, ci, vals = oracle.assemble(m.dofmap, A, m.n_dofs)
    K = sp.csr_matrix((vals, ci, rp), shape=(m.n_dofs, m.n_dofs))
    u = _hex_nodal(m, 2, lambda x: x[:, 0] ** 2 * x[:, 1])
    v = _hex_nodal(m, 2, lambda x: x[:, 1] * x[:, 2])
    assert abs(u @ (K @ v) - 1.0 / 6.0) < 1e-14


@pytest.mark.parametrize("mistake", ["swap_slabs", "flip_sign", "points_reordered"])
def test_stiffness_pins_are_sharp(mistake, monkeypatch):
    """Plausible mistakes planted in the oracle's inputs break a pin: two
    derivative slabs exchanged, one slab's sign flipped (both invisible on
    the unit cube, where G is diagonal and the sum symmetric in the axes),
    and quadrature points out of step with their weights."""
    tab, rule = H.tabulate, H.tensor_rule
    if mistake == "swap_slabs":
        monkeypatch.setattr(H, "tabulate", lambda p, X: (tab(p, X)[0], tab(p, X)[1][[1, 0, 2]]))
    elif mistake == "flip_sign":
        monkeypatch.setattr(H, "tabulate",
                            lambda p, X: (tab(p, X)[0], tab(p, X)[1] * np.array([1, 1, -1])[:, None, None]))
    else:
        def bad_rule(q):
            pts, w = rule(q)
            return np.roll(pts, 1, axis=0), w
        monkeypatch.setattr(H, "tensor_rule", bad_rule)
    m = hex_mesh(3, 2, jitter=0.25, seed=4)
    rows, energy, sym = _stiffness_pins(m, 2, 4)
    mu = hex_mesh(2, 2, jitter=0.0)
    A = H.stiffness_matrices(mu.cell_coords, 2, 4)
    rp, ci, vals = oracle.assemble(mu.dofmap, A, mu.n_dofs)
    K = sp.csr_matrix((vals, ci, rp), shape=(mu.n_dofs, mu.n_dofs))
    u = _hex_nodal(mu, 2, lambda x: x[:, 0] ** 2 * x[:, 1])
    v = _hex_nodal(mu, 2, lambda x: x[:, 1] * x[:, 2])
    poly = abs(u @ (K @ v) - 1.0 / 6.0)
    assert energy > 1e-6 or poly > 1e-6, (mistake, energy, poly)
