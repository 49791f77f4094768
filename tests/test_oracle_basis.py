"""Pins for the oracle's product-form Lagrange basis (not the GPU path)."""
from math import comb

import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("d,p,n", [(2, 1, 3), (3, 1, 4), (3, 4, 35), (3, 6, 84), (3, 8, 165), (2, 5, 21)])
def test_dimension(d, p, n):
    assert basis.n_phi(d, p) == n == comb(p + d, d)
    assert basis.multi_indices(d, p).shape == (n, d)


@pytest.mark.parametrize("d,p", [(2, 1), (2, 3), (3, 1), (3, 2), (3, 4), (3, 6)])
def test_kronecker_property(d, p):
    nodes = basis.multi_indices(d, p) / p
    vals, _ = basis.tabulate(d, p, nodes)
    np.testing.assert_allclose(vals, np.eye(len(nodes)), atol=1e-12)


def _random_points(d, n, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.dirichlet(np.ones(d + 1), size=n)[:, 1:]
    return x


@pytest.mark.parametrize("d,p", [(2, 2), (3, 3), (3, 4), (3, 6), (3, 8)])
def test_partition_of_unity_and_linear_reproduction(d, p):
    X = _random_points(d, 40)
    vals, grads = basis.tabulate(d, p, X)
    np.testing.assert_allclose(vals.sum(axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(grads.sum(axis=2), 0.0, atol=1e-10)
    nodes = basis.multi_indices(d, p) / p
    np.testing.assert_allclose(vals @ nodes, X, atol=1e-12)
    # gradient of sum_a X_a phi_a = identity
    for s in range(d):
        np.testing.assert_allclose(grads[s] @ nodes[:, s], 1.0, atol=1e-10)


def test_p1_is_barycentric():
    X = _random_points(3, 20, seed=1)
    vals, grads = basis.tabulate(3, 1, X)
    lam = np.concatenate([1 - X.sum(axis=1, keepdims=True), X], axis=1)
    np.testing.assert_allclose(vals, lam, atol=1e-15)
    np.testing.assert_allclose(grads[:, 0, :], [[-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]], atol=0)


@pytest.mark.parametrize("d,p", [(2, 3), (3, 4), (3, 6)])
def test_gradient_against_central_differences(d, p):
    X = _random_points(d, 10, seed=2) * 0.9 + 0.02
    _, grads = basis.tabulate(d, p, X)
    h = 1e-6
    for s in range(d):
        e = np.zeros(d); e[s] = h
        vp, _ = basis.tabulate(d, p, X + e)
        vm, _ = basis.tabulate(d, p, X - e)
        np.testing.assert_allclose(grads[s], (vp - vm) / (2 * h), atol=5e-6 * p ** 2)
