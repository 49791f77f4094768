"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (from the method's error analysis and the workload targets):
  * FP64 path: every entry within 1e-12 * max|A| of the oracle (normwise
    relative 1e-12); CSR row_ptr / col_idx bit-identical.
  * FP16 storage and H formation, FP32 accumulation: relative Frobenius
    error <= 1e-3.
  * split FP16 (hi + lo), FP32 accumulation: <= 1e-6.
  * FP32: <= 1e-5 (storage and accumulation in single: a few u_32 = 6e-8
    times the cancellation factor kappa_q of Corollary 4.10, measured <= 50
    here; 1e-5 leaves margin for K = 1536 accumulations).
  * BF16 storage: no normwise bar of its own (u_bf16 = 3.9e-3 is above the
    1e-3 target); held, like every mixed mode, to the entrywise bound below.
Every mixed mode is also held entrywise, on every CSR entry of the small
meshes, to the rounding error bound of the analysis (Theorem 4.8 /
Corollary 4.10, see U_S and _bound_csr).  Floating-point results of mixed
modes are compared by tolerance only; the summation order inside a
matrix-core instruction is hardware-defined.  At the full benchmark sizes,
sampled rows are held to the same entrywise bound (see _row_bound).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from fe_inputs import config_mesh
from paper_2410_12614_amd import _lib as L
from paper_2410_12614_amd import api

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp16": 1e-3, "split": 1e-6, "fp32": 1e-5, "bf16": None}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()   # raises if libfe.so is missing: no fallback
    yield
    torch.cuda.synchronize()


def run_assembly(mesh, forms, prec, q, coeff=None, gather=False):
    descs = [api.form_desc(mesh.d, mesh.degree, q, f, prec, has_coeff=coeff is not None) for f in forms]
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs, coeff)
    asm = api.Assembly(mv, descs)
    vals = asm.numeric(gather=gather)
    torch.cuda.synchronize()
    st = asm.status()
    return asm, [v[:asm.nnz].double().cpu().numpy() for v in vals], st


_ORACLE = {}


def oracle_csr(key, mesh, form, q, coeff=None):
    k = (key, form)
    if k not in _ORACLE:
        A = oracle.local_matrices(form, mesh.cell_coords, mesh.degree, q, mesh.dofmap, coeff)
        _ORACLE[k] = oracle.assemble(mesh.dofmap, A, mesh.n_dofs) + (A,)
    return _ORACLE[k]


CASES = {
    # name: (mesh builder, forms, q, with coefficient)
    "c1": (lambda: config_mesh("c1"), ("stiffness",), 0, False),
    "c2s": (lambda: config_mesh("c2", n=3), ("mass", "stiffness"), 8, False),
    "c3s": (lambda: config_mesh("c3", n=2), ("stiffness",), 14, True),
}
_MESH = {}


def mesh_of(name):
    if name not in _MESH:
        _MESH[name] = CASES[name][0]()
    return _MESH[name]


# c1 is the FP64 correctness configuration; the mixed modes run on c2s, c3s
PARITY = [(n, p, path) for n in ("c1", "c2s", "c3s")
          for p in ("fp64", "fp16", "split", "fp32", "bf16")
          for path in ("numeric", "gather") if n != "c1" or p == "fp64"]


@pytest.mark.parametrize("name,prec,path", PARITY)
def test_assembly_parity(name, prec, path):
    mesh = mesh_of(name)
    _, forms, q, has_c = CASES[name]
    coeff = mesh.coeff if has_c else None
    say(f"[parity] {name} {prec} {path} cells={mesh.n_cells} p={mesh.degree} q={q}")
    asm, vals, st = run_assembly(mesh, forms, prec, q, coeff, gather=(path == "gather"))
    assert all(s == 0 for s in st), st
    for f, v in zip(forms, vals):
        rp, ci, ref, _ = oracle_csr(name, mesh, f, q, coeff)
        np.testing.assert_array_equal(asm.row_ptr.cpu().numpy(), rp)
        np.testing.assert_array_equal(asm.col_idx[:asm.nnz].cpu().numpy(), ci)
        scale = np.abs(ref).max()
        if prec == "fp64":
            err = np.abs(v - ref).max() / scale
        else:
            err = np.linalg.norm(v - ref) / np.linalg.norm(ref)
            ratio = _entrywise_ratio(mesh, f, q, coeff, prec, v, ref)
            say(f"[parity] {name} {prec} {path} {f}: error / entrywise bound <= {ratio:.3f}")
            assert ratio <= 2.0, (name, prec, f, ratio)
        say(f"[parity] {name} {prec} {path} {f}: err {err:.3e} (bar {TOL[prec]})")
        if TOL[prec] is not None:
            assert err <= TOL[prec], (name, prec, f, err)


@pytest.mark.parametrize("p,q", [(1, 2), (2, 4), (3, 6), (5, 10), (7, 14), (8, 16)])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_all_degrees_local_matrices(p, q, prec):
    """Every tile instantiation (row tiles 1, 2, 4, 8, 11) against the oracle's
    element matrices, through fe_cell_kernels."""
    mesh = config_mesh("c2", n=2 if p <= 5 else 1, degree=p)
    say(f"[local] p={p} q={q} {prec} cells={mesh.n_cells}")
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    for form in ("mass", "stiffness"):
        desc = api.form_desc(3, p, q, form, prec)
        buf = api.fe_form_prepare(desc)
        n_phi = mesh.n_phi
        dt = torch.float64 if prec == "fp64" else torch.float32
        A = torch.full((mesh.n_cells, n_phi, n_phi), float("nan"), dtype=dt, device="cuda")
        api.fe_cell_kernels(desc, buf, mv, A)
        torch.cuda.synchronize()
        assert api.fe_get_device_status(buf) == 0
        ref = oracle.local_matrices(form, mesh.cell_coords, p, q)
        got = A.double().cpu().numpy()
        if prec == "fp64":
            err = max(np.abs(got[c] - ref[c]).max() / np.abs(ref[c]).max() for c in range(mesh.n_cells))
        else:
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"[local] p={p} {prec} {form}: err {err:.3e}")
        assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp16", "split", "fp32", "bf16"])
@pytest.mark.parametrize("p,q", [(2, 4), (4, 8), (5, 10)])
def test_fused_equals_gather_bitwise(prec, p, q):
    """The fused row-ownership path and the cell-kernel + row-gather path sum
    every entry in the same order (cell ascending) from the same matrix-core
    columns, so their values agree bit for bit (local rows longer than 64
    entries: the Q4 hexahedral case of the hexahedral tests)."""
    mesh = config_mesh("c2", n=3 if p < 5 else 2, degree=p)
    descs = [api.form_desc(3, p, q, f, prec) for f in ("mass", "stiffness")]
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    asm = api.Assembly(mv, descs)
    assert 0 < asm.max_row_len <= 1024
    a = [v.clone() for v in asm.numeric()]
    b = asm.numeric(gather=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        diff = (x != y).sum().item()
        say(f"[fused=gather] p={p} {prec}: {diff} differing entries of {x.numel()}")
        assert torch.equal(x, y)


def test_numeric_is_bitwise_repeatable():
    mesh = mesh_of("c2s")
    descs = [api.form_desc(3, 4, 8, f, "fp16") for f in ("mass", "stiffness")]
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    asm = api.Assembly(mv, descs)
    a = [v.clone() for v in asm.numeric()]
    b = asm.numeric()
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("prec,forms", [("fp16", ("mass", "stiffness")), ("fp64", ("mass",))])
def test_numeric_halves_equal_numeric(prec, forms):
    """FE_NUMERIC_GEOMETRY then FE_NUMERIC_FUSED (twice, the second reusing
    the records) give exactly the values of FE_NUMERIC; the halves are
    refused where the fused path does not apply (a coefficient form, or
    FP64 stiffness, whose tables do not fit on chip)."""
    mesh = mesh_of("c2s")
    descs = [api.form_desc(3, 4, 8, f, prec) for f in forms]
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    asm = api.Assembly(mv, descs)
    ref = [v.clone() for v in asm.numeric()]
    for v in asm.values:
        v.fill_(float("nan"))
    asm.numeric(part="geometry")
    for _ in range(2):
        got = asm.numeric(part="fused")
        torch.cuda.synchronize()
        for x, y in zip(ref, got):
            assert torch.equal(x, y)
    mesh3 = mesh_of("c3s")
    mv3 = api.MeshView.from_numpy(mesh3.cell_coords, mesh3.dofmap, mesh3.n_dofs, mesh3.coeff)
    asm3 = api.Assembly(mv3, [api.form_desc(3, 6, 14, "stiffness", prec, has_coeff=True)])
    with pytest.raises(L.FeError) as e:
        asm3.numeric(part="fused")
    assert e.value.status == L.FE_EUNSUPPORTED
    if prec == "fp64":
        asm_k = api.Assembly(mv, [api.form_desc(3, 4, 8, "stiffness", "fp64")])
        with pytest.raises(L.FeError) as e:
            asm_k.numeric(part="geometry")
        assert e.value.status == L.FE_EUNSUPPORTED


def test_degenerate_cell_sets_status_and_nan():
    mesh = config_mesh("c2", n=1, degree=2, flatten=0.0)
    coords = mesh.cell_coords.copy()
    coords[3, 3] = coords[3, 0] + 0.5 * (coords[3, 1] - coords[3, 0])   # det J = 0
    mv = api.MeshView.from_numpy(coords, mesh.dofmap, mesh.n_dofs)
    desc = api.form_desc(3, 2, 4, "stiffness", "fp16")
    buf = api.fe_form_prepare(desc)
    A = torch.zeros((mesh.n_cells, 10, 10), dtype=torch.float32, device="cuda")
    api.fe_cell_kernels(desc, buf, mv, A)
    torch.cuda.synchronize()
    assert api.fe_get_device_status(buf) == L.FE_EDEGENERATE
    assert api.fe_get_device_status(buf) == 0          # read-and-clear
    An = A.cpu().numpy()
    assert np.isnan(An[3]).all()
    assert np.isfinite(np.delete(An, 3, axis=0)).all()


def test_empty_mesh_is_a_no_op():
    desc = api.form_desc(3, 4, 8, "mass", "fp16")
    buf = api.fe_form_prepare(desc)
    mv = api.MeshView(torch.zeros((0, 4, 3), dtype=torch.float64, device="cuda"),
                      torch.zeros((0, 35), dtype=torch.int32, device="cuda"), 10)
    api.fe_cell_kernels(desc, buf, mv, torch.zeros(1, device="cuda"))
    torch.cuda.synchronize()


def test_bad_dof_is_reported():
    mesh = config_mesh("c2", n=1, degree=2, flatten=0.0)
    dm = mesh.dofmap.copy()
    dm[2, 4] = mesh.n_dofs + 7
    mv = api.MeshView.from_numpy(mesh.cell_coords, dm, mesh.n_dofs)
    descs = [api.form_desc(3, 2, 4, "mass", "fp64")]
    with pytest.raises(L.FeError) as e:
        api.Assembly(mv, descs)
    assert e.value.status == L.FE_EINVAL


# Entrywise rounding-error bound of the mixed modes (Theorem 4.8 /
# Corollary 4.10): |A_hat - A| <= (k_s u_s + (n_d^2 + n_q) u_q) M + M_g with
# M = sum_s sum_t |B_s|^T |C_st| |B_t|, assembled, and M_g the geometry term
# (the FP64 geometry's own rounding error in place of |C_st|).  k_s counts the roundings
# at the storage precision: B and H (k_s = 2), plus, when H is formed in half
# arithmetic from a half weighted table and half geometry factors, those two
# roundings and the three rounded steps of the sum over t (k_s = 7).
U_S = {"fp16": (7, 2.0 ** -11), "bf16": (2, 2.0 ** -8), "split": (2, 2.0 ** -22),
       "fp32": (2, 2.0 ** -24)}
U_Q = 2.0 ** -24


U_G = 2.0 ** -53


def _geometry_abs(x, form):
    """(|G|, dG) of one cell: the geometry tensor and the rounding error of
    its FP64 evaluation (the u_g term of Corollary 4.10), every entry of G
    off by at most a few u_g kappa(J) max|G| -- so that entries of G that are
    exactly zero (cells aligned with the axes) still get an absolute bound."""
    J, det, Ji, G = oracle.geometry(x)
    if form == "mass":
        return np.array([[abs(det)]]), np.array([[8 * U_G * abs(det)]])
    kappa = np.linalg.norm(J) * np.linalg.norm(Ji)
    return np.abs(G), np.full(G.shape, 16 * U_G * kappa * np.abs(G).max())


def _cell_bound(B, w, z, Gabs, i):
    """sum_s sum_t sum_q |B_s(q, i)| w_q |z_q| |G_st| |B_t(q, :)| of one cell."""
    left = Gabs @ np.abs(B[:, :, i])                           # [t][q]
    return np.einsum("tq,tqj->j", left * (w * z)[None, :], np.abs(B))


_BOUND = {}


def _bound_csr(mesh, form, q, coeff):
    """(M, M_g): M = sum_K L_K (sum_s sum_t |B_s|^T |C_st| |B_t|) L_K^T in CSR
    order (the oracle's pattern), and M_g the same sum with |C_st| replaced by
    the geometry rounding error, for the entrywise bound of the mixed modes."""
    key = (id(mesh), form, q, coeff is not None)
    if key not in _BOUND:
        _BOUND[key] = _bound_csr_uncached(mesh, form, q, coeff)
    return _BOUND[key]


def _bound_csr_uncached(mesh, form, q, coeff):
    _, w, vals, grads = oracle.tabulation(mesh.d, mesh.degree, q)
    B = vals[None] if form == "mass" else grads
    Ml = np.zeros((mesh.n_cells, mesh.n_phi, mesh.n_phi))
    Mg = np.zeros_like(Ml)
    for K in range(mesh.n_cells):
        Gabs, dG = _geometry_abs(mesh.cell_coords[K], form)
        z = np.abs(vals @ coeff[mesh.dofmap[K]]) if coeff is not None else np.ones(len(w))
        for i in range(mesh.n_phi):
            Ml[K, i] = _cell_bound(B, w, z, Gabs, i)
            Mg[K, i] = _cell_bound(B, w, z, dG, i)
    return (oracle.assemble(mesh.dofmap, Ml, mesh.n_dofs)[2],
            oracle.assemble(mesh.dofmap, Mg, mesh.n_dofs)[2])


def _entrywise_ratio(mesh, form, q, coeff, prec, got, ref):
    """max over CSR entries of |got - ref| / bound (entries with a zero bound
    must be exact)."""
    k_s, u_s = U_S[prec]
    nd = 1 if form == "mass" else mesh.d
    n_q = len(oracle.tabulation(mesh.d, mesh.degree, q)[1])
    M, Mg = _bound_csr(mesh, form, q, coeff)
    bound = (k_s * u_s + (nd * nd + n_q) * U_Q) * M + Mg
    err = np.abs(got - ref)
    return float(np.where(bound > 0, err / np.where(bound > 0, bound, 1.0),
                          np.where(err > 0, np.inf, 0.0)).max())


def _row_bound(mesh, form, q, coeff, g, cells, cols):
    """(M, M_g) restricted to CSR row g, ordered like cols."""
    _, w, vals, grads = oracle.tabulation(mesh.d, mesh.degree, q)
    B = vals[None] if form == "mass" else grads                 # [s][q][k]
    M, Mg = {}, {}
    for K in cells:
        Gabs, dG = _geometry_abs(mesh.cell_coords[K], form)
        z = np.abs(vals @ coeff[mesh.dofmap[K]]) if coeff is not None else np.ones(len(w))
        i = int(np.nonzero(mesh.dofmap[K] == g)[0][0])
        Mi = _cell_bound(B, w, z, Gabs, i)
        Mgi = _cell_bound(B, w, z, dG, i)
        for j in range(mesh.n_phi):
            h = int(mesh.dofmap[K, j])
            M[h] = M.get(h, 0.0) + Mi[j]
            Mg[h] = Mg.get(h, 0.0) + Mgi[j]
    return np.array([M[h] for h in cols]), np.array([Mg[h] for h in cols])


def _sampled_rows_check(mesh, forms, prec, q, coeff, rows, asm, vals):
    """Rows computed one by one by the oracle.  FP64: every entry within
    1e-12 max|row|.  Mixed modes: every entry within the rounding-error
    bound above (with a 2x margin for the O(u^2) terms)."""
    rp = asm.row_ptr.cpu().numpy()
    ci_all = asm.col_idx[:asm.nnz]
    for g in rows:
        cells = np.nonzero((mesh.dofmap == g).any(axis=1))[0]
        for f, v in zip(forms, vals):
            A = oracle.local_matrices(f, mesh.cell_coords[cells], mesh.degree, q,
                                      mesh.dofmap[cells], coeff)
            ref = {}
            for c_i, K in enumerate(cells):
                i = int(np.nonzero(mesh.dofmap[K] == g)[0][0])
                for j in range(mesh.n_phi):
                    h = int(mesh.dofmap[K, j])
                    ref[h] = ref.get(h, 0.0) + A[c_i, i, j]
            cols = ci_all[rp[g]:rp[g + 1]].cpu().numpy()
            assert sorted(ref) == list(cols)
            r = np.array([ref[h] for h in cols])
            got = v[rp[g]:rp[g + 1]]
            if prec == "fp64":
                err = np.abs(got - r).max() / np.abs(r).max()
                assert err <= TOL["fp64"], (g, f, err)
            else:
                k_s, u_s = U_S[prec]
                nd = 1 if f == "mass" else mesh.d
                n_q = len(oracle.tabulation(mesh.d, mesh.degree, q)[1])
                M, Mg = _row_bound(mesh, f, q, coeff, g, cells, cols)
                bound = (k_s * u_s + (nd * nd + n_q) * U_Q) * M + Mg
                err = np.abs(got - r)
                # an entry whose bound is zero (no nonzero terms) must be exact
                ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0),
                                 np.where(err > 0, np.inf, 0.0)).max()
                assert ratio <= 2.0, (g, f, ratio)


@pytest.mark.parametrize("prec", ["fp16", "fp64", "split"])
def test_full_size_c2_sampled_rows(prec):
    """The benchmark workload (82,944 P4 cells, mass + stiffness) in the
    launch configuration the benchmark times: pattern size and sortedness,
    and 24 seeded rows (including rows of flattened cells) against the
    oracle computed row by row, within the entrywise error bound."""
    mesh = config_mesh("c2")
    say(f"[full c2] {prec}")
    asm, vals, st = run_assembly(mesh, ("mass", "stiffness"), prec, 8)
    assert all(s == 0 for s in st)
    assert asm.nnz == 67338433
    rp = asm.row_ptr.cpu().numpy()
    assert rp[0] == 0 and np.all(np.diff(rp) > 0)
    ci = asm.col_idx[:asm.nnz]
    seg = torch.from_numpy(np.repeat(np.arange(mesh.n_dofs), np.diff(rp))).cuda()
    d = ci[1:] - ci[:-1]
    same = seg[1:] == seg[:-1]
    assert bool(((d > 0) | ~same).all())
    rng = np.random.default_rng(5)
    rows = list(rng.choice(mesh.n_dofs, 16, replace=False))
    rows += list(np.unique(mesh.dofmap[mesh.flattened[:4]].ravel())[:8])
    _sampled_rows_check(mesh, ("mass", "stiffness"), prec, 8, None, rows, asm, vals)


_C3 = {}


@pytest.mark.parametrize("prec", ["fp16", "fp64", "bf16", "fp32", "split"])
def test_full_size_c3_sampled_rows(prec):
    """The weighted-stiffness workload at full size (196,608 P6 cells, 512
    quadrature points, FE coefficient) in every precision, in the launch
    configuration the benchmark times: pattern size and sortedness, and 12
    seeded rows against the oracle computed row by row (only those rows are
    copied back), FP64 to 1e-12 and the mixed modes within the entrywise
    rounding error bound."""
    if "mesh" not in _C3:
        _C3["mesh"] = config_mesh("c3")
    mesh = _C3["mesh"]
    say(f"[full c3] {prec}")
    desc = api.form_desc(3, 6, 14, "stiffness", prec, has_coeff=True)
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs, mesh.coeff)
    asm = api.Assembly(mv, [desc])
    (vals,) = asm.numeric()
    torch.cuda.synchronize()
    assert all(s == 0 for s in asm.status())
    assert asm.nnz == 1094564353
    rp_d = asm.row_ptr
    assert int(rp_d[0]) == 0 and bool((rp_d[1:] > rp_d[:-1]).all())
    rp = rp_d.cpu().numpy()
    rng = np.random.default_rng(7)
    rows = [int(g) for g in rng.choice(mesh.n_dofs, 12, replace=False)]

    picked = []
    for g in rows:
        seg = asm.col_idx[rp[g]:rp[g + 1]]
        assert bool((seg[1:] > seg[:-1]).all())
        picked.append(vals[rp[g]:rp[g + 1]].double().cpu().numpy())
    full = {g: v for g, v in zip(rows, picked)}

    class V:      # CSR values view that serves only the sampled rows
        def __getitem__(self, sl):
            g = int(np.searchsorted(rp, sl.start, side="right") - 1)
            assert rp[g] == sl.start and rp[g + 1] == sl.stop
            return full[g]

    _sampled_rows_check(mesh, ("stiffness",), prec, 14, mesh.coeff, rows, asm, [V()])
