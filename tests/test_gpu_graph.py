"""FE_NUMERIC captured in one HIP graph (Assembly.capture / replay): every
replay, with eager work and synchronisations between the replays, gives the
bits of the eager call, for the fused path in FP16 and FP64 and for the
gather path of a coefficient form."""
import sys

import pytest
import torch

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


def _replays_match(asm, **kw):
    ref = [v[:asm.nnz].clone() for v in asm.numeric(**kw)]
    asm.capture(**kw)
    for r in range(3):
        for v in asm.values:
            v.fill_(float("nan"))            # eager work between the replays
        torch.cuda.synchronize()
        got = asm.replay()
        torch.cuda.synchronize()
        for f, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a[:asm.nnz], b), (r, f)
        assert all(s == 0 for s in asm.status())
    # an eager call after the replays still gives the same bits
    for a, b in zip(asm.numeric(**kw), ref):
        assert torch.equal(a[:asm.nnz], b)


@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_fused_numeric_graph_replays_match_eager(prec):
    m = config_mesh("c2", n=4, degree=4)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
    asm = api.Assembly(mv, [api.form_desc(3, 4, 8, f, prec) for f in ("mass", "stiffness")])
    _replays_match(asm)
    say(f"[graph] c2 n=4 {prec}: {asm.nnz} entries, 3 replays bitwise equal to the eager pass")


def test_gather_numeric_graph_replays_match_eager():
    m = config_mesh("c3", n=3, degree=6)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs, m.coeff)
    asm = api.Assembly(mv, [api.form_desc(3, 6, 14, "stiffness", "fp16", has_coeff=True)])
    _replays_match(asm)


def test_capture_refuses_an_own_stream():
    m = config_mesh("c2", n=1, degree=1)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
    asm = api.Assembly(mv, [api.form_desc(3, 1, 2, "mass", "fp16")], stream=torch.cuda.Stream())
    with pytest.raises(ValueError):
        asm.capture()
