"""The allocation-free numeric entry point (fe_assemble_csr_noalloc) against
FE_NUMERIC of fe_assemble_csr: the same fused kernels, so the values agree
bit for bit; two calls in a row, the second on a smaller mesh (the scratch
array keeps the first call's records and must not leak into the second);
and its host-side refusals (a mesh whose records exceed the scratch array,
a form off the fused path), which enqueue nothing."""
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


def _assembly(n, prec, forms):
    mesh = config_mesh("c2", n=n)
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    asm = api.Assembly(mv, [api.form_desc(3, 4, 8, f, prec) for f in forms])
    return mesh, asm


# forms on the fused path: the FP16 mass + stiffness pair, FP64 mass (the
# FP64 Poisson tables do not fit on chip: that form takes the gather)
@pytest.mark.parametrize("prec,forms", [("fp16", ("mass", "stiffness")), ("fp64", ("mass",))])
def test_noalloc_equals_numeric_twice_second_smaller(prec, forms):
    for n in (4, 2):
        mesh, asm = _assembly(n, prec, forms)
        say(f"[noalloc] {prec} n={n}: {mesh.n_cells} cells, nnz {asm.nnz}")
        ref = [v[:asm.nnz].clone() for v in asm.numeric()]
        for v in asm.values:
            v.fill_(float("nan"))
        got = asm.numeric_noalloc()
        torch.cuda.synchronize()
        assert all(s == 0 for s in asm.status())
        for a, b in zip(ref, got):
            assert torch.equal(a, b[:asm.nnz])
        # and against the oracle, to the bar of the precision
        for f, v in zip(forms, got):
            _, _, want = oracle.assemble_form(f, mesh, 8)
            g = v[:asm.nnz].double().cpu().numpy()
            if prec == "fp64":
                err = np.abs(g - want).max() / np.abs(want).max()
                assert err <= 1e-12, (f, err)
            else:
                err = np.linalg.norm(g - want) / np.linalg.norm(want)
                assert err <= 1e-3, (f, err)


def test_noalloc_refusals():
    # the full P4 workload's records fit (82,944 cells); the P6 coefficient
    # form does not take the fused path
    m3 = config_mesh("c3", n=1)
    mv3 = api.MeshView.from_numpy(m3.cell_coords, m3.dofmap, m3.n_dofs, m3.coeff)
    asm3 = api.Assembly(mv3, [api.form_desc(3, 6, 14, "stiffness", "fp16", has_coeff=True)])
    with pytest.raises(L.FeError) as e:
        asm3.numeric_noalloc()
    assert e.value.status == L.FE_EUNSUPPORTED
    _, asm64 = _assembly(2, "fp64", ("mass", "stiffness"))
    with pytest.raises(L.FeError) as e:
        asm64.numeric_noalloc()
    assert e.value.status == L.FE_EUNSUPPORTED
    # more cells than the scratch array holds records for: refused on the host
    big = config_mesh("c2", n=40, degree=1)   # 384,000 P1 cells, two forms of 64 B records
    mvb = api.MeshView.from_numpy(big.cell_coords, big.dofmap, big.n_dofs)
    asmb = api.Assembly(mvb, [api.form_desc(3, 1, 2, f, "fp64") for f in ("mass", "stiffness")])
    if asmb.mats[0].schedule > 0:
        with pytest.raises(L.FeError) as e:
            asmb.numeric_noalloc()
        assert e.value.status == L.FE_ESIZE
