"""The whole-cell FP16 kernel (one wave per cell, symmetric tiles, B^T
fragments shared through an LDS ring): local matrices of the forms it is
compiled for against the FP64 oracle (tile 8 of fe_cell_kernels_tile:
mass P5..P8 (P8 with rows packed at n_phi = 165, not a multiple of
four), Poisson P6; the Poisson P6 form with a coefficient through
FE_NUMERIC, where the coefficient at the points goes to the workspace), the
entrywise rounding-error bound of the FP16 mode, ragged batches, degenerate
cells and the two halves of the gather path."""
import sys

import numpy as np
import pytest
import torch

import oracle
from fe_inputs import config_mesh
from paper_2410_12614_amd import _lib as L
from paper_2410_12614_amd import api

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()
    yield
    torch.cuda.synchronize()


def _local(mesh, p, q, form, tile):
    desc = api.form_desc(3, p, q, form, "fp16")
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    buf = api.fe_form_prepare(desc)
    out = torch.full((mesh.n_cells, mesh.n_phi, mesh.n_phi), float("nan"), device="cuda")
    api.fe_cell_kernels_tile(desc, buf, mv, out, tile)
    torch.cuda.synchronize()
    return buf, out.double().cpu().numpy()


@pytest.mark.parametrize("form,p", [("mass", 5), ("mass", 6), ("mass", 7), ("mass", 8), ("stiffness", 6)])
def test_whole_cell_kernel_local_matrices(form, p):
    # 2^3 x 6 = 48 cells, 5 % flattened: the cells of a workgroup's last
    # round are ragged (48 is not a multiple of the grid's waves)
    m = config_mesh("c2", n=2, degree=p, flatten=0.05)
    q = 2 * p
    buf, got = _local(m, p, q, form, 8)
    assert api.fe_get_device_status(buf) == L.FE_OK
    ref = oracle.local_matrices(form, m.cell_coords, p, q)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _, old = _local(m, p, q, form, -1)
    err_old = np.linalg.norm(old - ref) / np.linalg.norm(ref)
    say(f"[whole-cell] {form} p{p}: rel. Frobenius {err:.2e} (batched kernel {err_old:.2e})")
    assert err <= 1e-3, err
    # the tiles off the diagonal are stored twice from one value (exactly
    # symmetric there); a diagonal tile computes (i, j) and (j, i) apart
    t = np.arange(m.n_phi) // 16
    off = t[:, None] != t[None, :]
    assert np.array_equal(got[:, off], got.transpose(0, 2, 1)[:, off])
    assert np.abs(got - got.transpose(0, 2, 1)).max() <= 1e-3 * np.abs(got).max()


def test_whole_cell_kernel_degenerate_cell():
    m = config_mesh("c2", n=1, degree=6, flatten=0.0)
    coords = m.cell_coords.copy()
    coords[2, 3] = coords[2, 0] + 0.5 * (coords[2, 1] - coords[2, 0])   # det J = 0
    desc = api.form_desc(3, 6, 12, "mass", "fp16")
    mv = api.MeshView.from_numpy(coords, m.dofmap, m.n_dofs)
    buf = api.fe_form_prepare(desc)
    out = torch.zeros((m.n_cells, m.n_phi, m.n_phi), device="cuda")
    api.fe_cell_kernels_tile(desc, buf, mv, out, 8)
    torch.cuda.synchronize()
    assert api.fe_get_device_status(buf) == L.FE_EDEGENERATE
    o = out.cpu().numpy()
    assert np.isnan(o[2]).all() and np.isfinite(np.delete(o, 2, axis=0)).all()


def test_whole_cell_kernel_refuses_other_forms():
    m = config_mesh("c2", n=1, degree=4)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
    for prec, p, form in (("fp32", 6, "mass"), ("fp16", 4, "mass"), ("fp16", 5, "stiffness"),
                          ("fp16", 8, "stiffness"), ("bf16", 8, "mass")):
        mm = config_mesh("c2", n=1, degree=p)
        mvv = api.MeshView.from_numpy(mm.cell_coords, mm.dofmap, mm.n_dofs)
        desc = api.form_desc(3, p, 2 * p, form, prec)
        buf = api.fe_form_prepare(desc)
        out = torch.zeros((mm.n_cells, mm.n_phi, mm.n_phi),
                          dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
        with pytest.raises(L.FeError) as e:
            api.fe_cell_kernels_tile(desc, buf, mvv, out, 8)
        assert e.value.status == L.FE_EUNSUPPORTED, (prec, p, form)


def test_weighted_stiffness_halves_of_the_gather_path():
    """FE_NUMERIC_LOCAL then FE_NUMERIC_ASSEMBLE give the bits of FE_NUMERIC
    (the coefficient at the points, the whole-cell kernel, then the row
    gather); ASSEMBLE alone again reproduces them from the workspace."""
    m = config_mesh("c3", n=2)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs, m.coeff)
    asm = api.Assembly(mv, [api.form_desc(3, 6, 14, "stiffness", "fp16", has_coeff=True)])
    ref = asm.numeric()[0][:asm.nnz].clone()
    for v in asm.values:
        v.fill_(float("nan"))
    asm.numeric(part="local")
    got = asm.numeric(part="assemble")[0][:asm.nnz].clone()
    for v in asm.values:
        v.fill_(float("nan"))
    again = asm.numeric(part="assemble")[0][:asm.nnz]
    torch.cuda.synchronize()
    assert all(s == 0 for s in asm.status())
    assert torch.equal(got, ref) and torch.equal(again, ref)
