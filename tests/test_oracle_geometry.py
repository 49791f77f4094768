"""Pins for the oracle's geometry (Section 4.2), not the GPU path."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eps_tetrahedron.json")


def eps_tet(eps):
    # vertex 0 is the paper's origin vertex; vertices 1..3 follow in the paper's order
    return np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [eps, 1, -1]], dtype=float)


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"])
def test_eps_tetrahedron_closed_forms(case):
    eps = case["eps"]
    J, det, Jinv, G = oracle.geometry(eps_tet(eps))
    printed = np.array([[1, 1, 0], [1, 0, 1], [eps, 1, -1]], dtype=float)
    np.testing.assert_array_equal(J, printed.T)
    assert abs(det - case["det_J"]) <= 1e-15 * np.linalg.cond(J, 1) * abs(case["det_J"])
    kappa = np.linalg.norm(printed, np.inf) * np.linalg.norm(Jinv.T, np.inf)
    assert abs(kappa - case["kappa_inf_printed"]) <= 1e-9 * case["kappa_inf_printed"]
    np.testing.assert_allclose(J @ Jinv, np.eye(3), atol=1e-15 * case["kappa_inf_printed"])


@pytest.mark.parametrize("eps", [1e-1, 1e-3])
def test_eps_tetrahedron_scaled_translated(eps):
    x = eps_tet(eps) * 3 ** -0.5 + np.array([1 / 3, 2 / 3, 4 / 3])
    J, det, Jinv, G = oracle.geometry(x)
    assert abs(det - eps * 3 ** -1.5) <= 1e-12 * eps
    J0, _, _, _ = oracle.geometry(eps_tet(eps))
    assert abs(np.linalg.cond(J) - np.linalg.cond(J0)) <= 1e-9 * np.linalg.cond(J0)


def test_reference_cell_identity():
    for d in (2, 3):
        x = np.vstack([np.zeros(d), np.eye(d)])
        J, det, Jinv, G = oracle.geometry(x)
        np.testing.assert_array_equal(J, np.eye(d))
        assert det == 1.0
        np.testing.assert_array_equal(G, np.eye(d))


def _random_cells(d, n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, d + 1, d))


@pytest.mark.parametrize("d", [2, 3])
def test_against_numpy_linalg(d):
    for x in _random_cells(d, 50, 3):
        J, det, Jinv, G = oracle.geometry(x)
        Jn = (x[1:] - x[0]).T
        np.testing.assert_allclose(J, Jn, atol=1e-15)
        assert abs(det - np.linalg.det(Jn)) <= 1e-13 * abs(det) * np.linalg.cond(Jn)
        Ji = np.linalg.inv(Jn)
        np.testing.assert_allclose(Jinv, Ji, rtol=0, atol=1e-12 * np.abs(Ji).max() * np.linalg.cond(Jn))
        Gn = abs(np.linalg.det(Jn)) * Ji @ Ji.T
        np.testing.assert_allclose(G, Gn, rtol=0, atol=1e-12 * np.abs(Gn).max() * np.linalg.cond(Jn))


@pytest.mark.parametrize("d", [2, 3])
def test_rigid_motion_invariance_and_dilation(d):
    rng = np.random.default_rng(4)
    for x in _random_cells(d, 10, 5):
        _, det, _, G = oracle.geometry(x)
        Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
        b = rng.normal(size=d)
        _, det2, _, G2 = oracle.geometry(x @ Q.T + b)
        assert abs(abs(det2) - abs(det)) <= 1e-12 * abs(det)
        np.testing.assert_allclose(G2, G, rtol=1e-10, atol=1e-10 * np.abs(G).max())
        a = 2.5
        _, det3, _, G3 = oracle.geometry(a * x)
        assert abs(det3 - a ** d * det) <= 1e-12 * abs(det3)
        np.testing.assert_allclose(G3, a ** (d - 2) * G, rtol=1e-12, atol=1e-12 * np.abs(G).max())


def test_degenerate_cell_raises():
    with pytest.raises(oracle.OracleError):
        oracle.geometry(eps_tet(0.0))
    x = eps_tet(0.5)
    x[2, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.geometry(x)
