"""Checks of the seeded input generators (meshes, dof maps, coefficient)."""
import numpy as np
import pytest

from fe_inputs import config_mesh, lattice_multi_indices


def signed_volumes(cc):
    e = cc[:, 1:, :] - cc[:, :1, :]
    return np.linalg.det(e)


@pytest.mark.parametrize("name,nk,nphi,ndofs", [("c1", 2048, 3, 1089), ("c2", 82944, 35, 912673)])
def test_config_counts(name, nk, nphi, ndofs):
    m = config_mesh(name)
    assert (m.n_cells, m.n_phi, m.n_dofs) == (nk, nphi, ndofs)
    assert m.dofmap.dtype == np.int32 and m.cell_coords.dtype == np.float64
    assert m.dofmap.min() == 0 and m.dofmap.max() == ndofs - 1
    # every local dof list is duplicate-free
    s = np.sort(m.dofmap, axis=1)
    assert np.all(np.diff(s, axis=1) > 0)


def test_c3_counts_small():
    m = config_mesh("c3", n=4)
    assert (m.n_cells, m.n_phi, m.n_dofs) == (6 * 64, 84, 25 ** 3)
    assert m.coeff is not None and np.all(m.coeff > np.exp(-1) - 1e-12) and np.all(m.coeff < np.e + 1e-12)


def test_jitter_keeps_orientation_and_is_seeded():
    from fe_inputs.meshes import kuhn_mesh
    for name in ("c1", "c2"):
        m = config_mesh(name, flatten=0.0)
        v0, cells, _ = kuhn_mesh(m.d, m.n)
        s0 = np.sign(signed_volumes(v0[cells]))
        s1 = np.sign(signed_volumes(m.cell_coords))
        assert np.all(s0 == s1) and np.all(s0 != 0)
        m2 = config_mesh(name, flatten=0.0)
        np.testing.assert_array_equal(m.cell_coords, m2.cell_coords)


def test_flattened_cells_have_aspect_1e3():
    m = config_mesh("c2", n=6)
    m0 = config_mesh("c2", n=6, flatten=0.0)
    assert len(m.flattened) == int(0.05 * m.n_cells)
    x = m.cell_coords[m.flattened]
    x0 = m0.cell_coords[m.flattened]
    base = x[:, 0]
    nrm = np.cross(x[:, 1] - base, x[:, 2] - base)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    alt = np.abs(np.einsum("ij,ij->i", x[:, 3] - base, nrm))
    longest = np.max([np.linalg.norm(x0[:, a] - x0[:, b], axis=1)
                      for a in range(4) for b in range(a + 1, 4)], axis=0)
    np.testing.assert_allclose(longest / alt, 1e3, rtol=1e-9)


def test_local_dof_order_p1_is_vertex_order():
    np.testing.assert_array_equal(lattice_multi_indices(3, 1), [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    m = config_mesh("c2", n=2, degree=1, flatten=0.0)
    np.testing.assert_array_equal(m.dofmap, m.cells)
