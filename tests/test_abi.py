"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side logic (tabulation, validation, size queries) is right.
No call here touches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2410_12614_amd import _lib as L
from paper_2410_12614_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2410_12614_amd import build
        build.build()
    return L.load()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.fe_version().startswith(b"fe-mi355x")


def test_status_strings(lib):
    for s in (L.FE_OK, L.FE_EINVAL, L.FE_EUNSUPPORTED, L.FE_EOVERFLOW, L.FE_EHIP,
              L.FE_EDEGENERATE, L.FE_ESIZE):
        assert lib.fe_status_string(s) != b"unknown status"
    assert lib.fe_status_string(12345) == b"unknown status"


@pytest.mark.parametrize("d,p,q", [(2, 1, 0), (2, 5, 10), (3, 1, 2), (3, 4, 8), (3, 6, 14), (3, 8, 16)])
def test_tabulate_matches_oracle(lib, d, p, q):
    pts, w, tab = api.fe_tabulate(d, p, q)
    opts, ow, ov, og = oracle.tabulation(d, p, q)
    np.testing.assert_allclose(pts, opts, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, ow, rtol=1e-13, atol=0)
    np.testing.assert_allclose(tab[0], ov, rtol=0, atol=5e-14)
    np.testing.assert_allclose(tab[1:], og, rtol=0, atol=1e-13 * np.abs(og).max())


@pytest.mark.parametrize("p,q", [(1, 2), (2, 4), (3, 6), (4, 8), (2, 0), (5, 10), (7, 14)])
def test_tabulate_hexahedron_matches_oracle(lib, p, q):
    import oracle.hexahedra as H
    pts, w, tab = api.fe_tabulate(L.FE_HEXAHEDRON, p, q)
    opts, ow = H.tensor_rule(q)
    ov, og = H.tabulate(p, opts)
    np.testing.assert_allclose(pts, opts, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, ow, rtol=1e-13, atol=0)
    np.testing.assert_allclose(tab[0], ov, rtol=0, atol=5e-14)
    np.testing.assert_allclose(tab[1:], og, rtol=0, atol=1e-13 * np.abs(og).max())


def test_tabulate_values_only_and_sizes(lib):
    n_phi, n_q = ctypes.c_int32(), ctypes.c_int32()
    assert lib.fe_tabulate(3, 6, 14, 0, ctypes.byref(n_phi), ctypes.byref(n_q), None, None, None) == 0
    assert (n_phi.value, n_q.value) == (84, 512)
    _, _, tab = api.fe_tabulate(3, 2, 4, nderiv=0)
    assert tab.shape == (1, 27, 10)


@pytest.mark.parametrize("args,status", [
    ((4, 1, 0, 1), L.FE_EINVAL),          # bad cell
    ((3, 0, 0, 1), L.FE_EINVAL),          # degree < 1
    ((3, 1, -1, 1), L.FE_EINVAL),         # negative quadrature degree
    ((3, 1, 0, 2), L.FE_EINVAL),          # nderiv not 0/1
    ((3, 9, 0, 1), L.FE_EUNSUPPORTED),    # degree > 8
    ((3, 2, 18, 1), L.FE_EUNSUPPORTED),   # quadrature degree > 17
])
def test_tabulate_errors(lib, args, status):
    n_phi, n_q = ctypes.c_int32(), ctypes.c_int32()
    assert lib.fe_tabulate(*args, ctypes.byref(n_phi), ctypes.byref(n_q), None, None, None) == status


def test_tabulate_null_size_pointers(lib):
    assert lib.fe_tabulate(3, 1, 0, 1, None, None, None, None, None) == L.FE_EINVAL


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "split"])
@pytest.mark.parametrize("d,p,q,form", [(3, 4, 8, "stiffness"), (3, 6, 14, "mass"), (2, 1, 0, "stiffness")])
def test_form_prepare_size_query(lib, prec, d, p, q, form):
    desc = api.form_desc(d, p, q, form, prec, has_coeff=(p == 6))
    sz = ctypes.c_size_t(0)
    assert lib.fe_form_prepare(ctypes.byref(desc), None, ctypes.byref(sz), None) == 0
    n_phi = oracle.basis.n_phi(d, p)
    m = q // 2 + 1
    n_q = m ** d
    elt = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2, "split": 4}[prec]
    nd = 1 if form == "mass" else d
    kstep = 32 if prec in ("fp16", "bf16", "split") else 4
    nqp = -(-n_q // kstep) * kstep
    mt = -(-n_phi // 16)
    assert sz.value >= mt * 16 * nd * nqp * elt      # at least the B^T operand
    assert sz.value < 64 << 20


@pytest.mark.parametrize("field,value,status", [
    ("cell", 5, L.FE_EINVAL), ("degree", 0, L.FE_EINVAL), ("degree", 9, L.FE_EUNSUPPORTED),
    ("form", 7, L.FE_EINVAL), ("precision", 9, L.FE_EINVAL), ("geom_precision", 3, L.FE_EINVAL),
    ("has_coeff", 3, L.FE_EINVAL), ("quad_degree", 18, L.FE_EUNSUPPORTED),
])
def test_form_validation(lib, field, value, status):
    desc = api.form_desc(3, 4, 8, "stiffness", "fp16")
    setattr(desc, field, value)
    sz = ctypes.c_size_t(0)
    assert lib.fe_form_prepare(ctypes.byref(desc), None, ctypes.byref(sz), None) == status


def _assemble_query(lib, descs, n_cells, n_dofs, plan=None):
    n = len(descs)
    darr = (L.fe_form_desc * max(n, 1))(*descs)
    mv = L.fe_mesh_view(n_cells=n_cells, cell_coords=None, dofmap=None, n_dofs=n_dofs, coeff=None)
    mats = (L.fe_csr * max(n, 1))()
    pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    st = lib.fe_assemble_csr(darr, None, n, ctypes.byref(mv), L.FE_NUMERIC, mats, plan,
                             ctypes.byref(pb), None, ctypes.byref(wb), None)
    return st, pb.value, wb.value


def test_assemble_size_query(lib):
    d1 = api.form_desc(3, 4, 8, "mass", "fp16")
    d2 = api.form_desc(3, 4, 8, "stiffness", "fp16")
    st, pb, wb = _assemble_query(lib, [d1, d2], 82944, 912673)
    assert st == 0
    # plan holds at least the 16-bit rank of every local entry
    assert pb >= 82944 * 35 * 35 * 2
    # workspace: FP32 local matrices of both forms (gather path) + per-form,
    # per-cell factor records (at most 64 bytes) of the fused path
    local = 2 * 82944 * 35 * 35 * 4
    assert wb == ((local + 255) // 256) * 256 + 2 * 64 * 82944


def test_assemble_size_query_hexahedra(lib):
    d = api.form_desc(L.FE_HEXAHEDRON, 4, 8, "mass", "fp16")
    n_cells, n_dofs = 54872, 3581577
    st, pb, wb = _assemble_query(lib, [d], n_cells, n_dofs)
    assert st == 0
    assert pb >= n_cells * 125 * 125 * 2
    # FP32 local matrices + factor records + the per-point factors (125
    # points padded to 128, at most 8 bytes each) of the fused halves
    a256 = lambda x: ((x + 255) // 256) * 256          # noqa: E731
    local = n_cells * 125 * 125 * 4
    assert wb == a256(local) + a256(64 * n_cells) + a256(n_cells * 128 * 8)


def test_assemble_argument_errors(lib):
    d1 = api.form_desc(3, 4, 8, "mass", "fp16")
    d2 = api.form_desc(3, 3, 8, "stiffness", "fp16")
    assert _assemble_query(lib, [], 10, 10)[0] == L.FE_EINVAL                    # no forms
    assert _assemble_query(lib, [d1] * 5, 10, 10)[0] == L.FE_EINVAL              # too many forms
    assert _assemble_query(lib, [d1, d2], 10, 10)[0] == L.FE_EINVAL              # degree mismatch
    d3 = api.form_desc(3, 4, 8, "stiffness", "fp64")
    assert _assemble_query(lib, [d1, d3], 10, 10)[0] == L.FE_EINVAL              # value type mismatch
    assert _assemble_query(lib, [d1], -1, 10)[0] == L.FE_EINVAL                  # negative cells
    assert _assemble_query(lib, [d1], 10, 0)[0] == L.FE_EINVAL                   # no dofs
    assert _assemble_query(lib, [d1], 10, 2 ** 31)[0] == L.FE_EOVERFLOW          # int32 columns


def test_cell_kernels_argument_errors(lib):
    desc = api.form_desc(3, 4, 8, "stiffness", "fp16", has_coeff=True)
    mv = L.fe_mesh_view(n_cells=10, cell_coords=None, dofmap=None, n_dofs=10, coeff=None)
    fake = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    assert lib.fe_cell_kernels(ctypes.byref(desc), None, ctypes.byref(mv), fake, None) == L.FE_EINVAL
    assert lib.fe_cell_kernels(ctypes.byref(desc), fake, ctypes.byref(mv), fake, None) == L.FE_EINVAL
    mv0 = L.fe_mesh_view(n_cells=0, cell_coords=None, dofmap=None, n_dofs=10, coeff=None)
    assert lib.fe_cell_kernels(ctypes.byref(desc), fake, ctypes.byref(mv0), None, None) == L.FE_OK


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of computing."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(L.FeLibraryError):
        api.fe_tabulate(3, 1, 0)


@pytest.mark.parametrize("span,elt", [(1024, 8), (2048, 4), (512, 4)])
def test_schedule_of_other_forms_is_rejected(lib, span, elt):
    """A fused schedule records the task span and value type of the forms it
    was built for; the fused half of the numeric phase refuses forms of
    another kind on the host, before anything is launched (the pointers
    below are never dereferenced)."""
    descs = [api.form_desc(3, 4, 8, f, "fp16") for f in ("mass", "stiffness")]
    darr = (L.fe_form_desc * 2)(*descs)
    fake = ctypes.c_void_p(4096)
    bufs = (ctypes.c_void_p * 2)(fake, fake)
    mv = L.fe_mesh_view(n_cells=82944, cell_coords=fake, dofmap=fake, n_dofs=912673, coeff=None)
    mats = (L.fe_csr * 2)()
    for m in mats:
        m.n_rows, m.nnz, m.schedule = 912673, 67338433, 1000
        m.schedule_span, m.schedule_elt = span, elt
        m.row_ptr = m.col_idx = m.values = 4096
    big = ctypes.c_size_t(1 << 62)
    for phase in (L.FE_NUMERIC_FUSED, L.FE_NUMERIC_GEOMETRY):
        st = lib.fe_assemble_csr(darr, bufs, 2, ctypes.byref(mv), phase, mats, fake,
                                 ctypes.byref(big), fake, ctypes.byref(big), None)
        assert st == L.FE_EINVAL, (phase, st)
