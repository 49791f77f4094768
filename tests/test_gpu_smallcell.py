"""The vector-ALU kernel of the smallest FP16 mass forms (tile 9 of
fe_cell_kernels_tile: P1, P2 tetrahedra, P1..P3 triangles): local matrices
against the FP64 oracle, against the batched matrix-core kernel (the same
half H, exact products summed in single in another order), ragged batches,
flattened and degenerate cells, and the forms it refuses."""
import sys

import numpy as np
import pytest
import torch

import oracle
from fe_inputs import config_mesh
from paper_2410_12614_amd import _lib as L
from paper_2410_12614_amd import api

pytestmark = pytest.mark.gpu

SMALL = 9


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()
    yield
    torch.cuda.synchronize()


def _local(m, p, q, tile, prec="fp16", form="mass", coords=None):
    desc = api.form_desc(m.d, p, q, form, prec)
    mv = api.MeshView.from_numpy(m.cell_coords if coords is None else coords, m.dofmap, m.n_dofs)
    buf = api.fe_form_prepare(desc)
    out = torch.full((m.cell_coords.shape[0], m.n_phi, m.n_phi), float("nan"), device="cuda")
    if tile < 0:
        api.fe_cell_kernels(desc, buf, mv, out)
    else:
        api.fe_cell_kernels_tile(desc, buf, mv, out, tile)
    torch.cuda.synchronize()
    return buf, out.double().cpu().numpy()


# (recipe, boxes, degree): 2 x 3^3 x 3 = 162 tetrahedra, 2 x 7^2 = 98
# triangles, neither a multiple of the 256 threads / n_phi rows of a
# workgroup; 5 % of the tetrahedra flattened by 10^3
@pytest.mark.parametrize("name,n,p", [("c2", 3, 1), ("c2", 3, 2), ("c1", 7, 1), ("c1", 7, 2), ("c1", 7, 3)])
def test_small_kernel_local_matrices(name, n, p):
    m = config_mesh(name, n=n, degree=p, flatten=0.05 if name == "c2" else 0.0)
    q = 2 * p
    buf, got = _local(m, p, q, SMALL)
    assert api.fe_get_device_status(buf) == L.FE_OK
    ref = oracle.local_matrices("mass", m.cell_coords, p, q)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _, mma = _local(m, p, q, -1)
    d_mma = np.abs(got - mma).max() / np.abs(mma).max()
    say(f"[small] {name} p{p}: {m.cell_coords.shape[0]} cells, rel. Frobenius {err:.2e}, "
        f"max diff to the matrix-core kernel {d_mma:.1e}")
    assert err <= 1e-3, err
    # the same H in half and exact products: only the order of the single
    # sums differs (n_q terms, a few units of 2^-24 of the largest entry;
    # forming H without its rounding to half would differ by about 2^-11)
    assert d_mma <= 1e-5, d_mma


def test_small_kernel_degenerate_cell():
    m = config_mesh("c2", n=2, degree=2, flatten=0.0)
    coords = m.cell_coords.copy()
    coords[5, 3] = coords[5, 0] + 0.25 * (coords[5, 1] - coords[5, 0])   # det J = 0
    buf, got = _local(m, 2, 4, SMALL, coords=coords)
    assert api.fe_get_device_status(buf) == L.FE_EDEGENERATE
    assert np.isnan(got[5]).all() and np.isfinite(np.delete(got, 5, axis=0)).all()


def test_small_kernel_refuses_other_forms():
    for name, prec, p, form in (("c2", "fp32", 2, "mass"), ("c2", "bf16", 1, "mass"),
                                ("c2", "fp16", 2, "stiffness"), ("c2", "fp16", 3, "mass"),
                                ("c1", "fp16", 4, "mass")):
        m = config_mesh(name, n=1, degree=p)
        desc = api.form_desc(m.d, p, 2 * p, form, prec)
        mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
        buf = api.fe_form_prepare(desc)
        out = torch.zeros((m.cell_coords.shape[0], m.n_phi, m.n_phi), device="cuda")
        with pytest.raises(L.FeError) as e:
            api.fe_cell_kernels_tile(desc, buf, mv, out, SMALL)
        assert e.value.status == L.FE_EUNSUPPORTED, (name, prec, p, form)
    # a tile past the last one is an argument error
    m = config_mesh("c2", n=1, degree=1)
    desc = api.form_desc(3, 1, 2, "mass", "fp16")
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
    buf = api.fe_form_prepare(desc)
    out = torch.zeros((m.cell_coords.shape[0], 4, 4), device="cuda")
    with pytest.raises(L.FeError) as e:
        api.fe_cell_kernels_tile(desc, buf, mv, out, 10)
    assert e.value.status == L.FE_EINVAL
