"""GPU parity of the actions (Algorithm 2) and their vector-Jacobian products
against the FP64 oracle, through the C ABI.

Bars:
  * FP64: every entry within 1e-12 * max|ref| of the oracle.
  * FP32 (tables, dofs, geometry factors and accumulation in single):
    relative 2-norm error <= 1e-4.  The analysis of the action (the theorem
    on the mixed-precision computation of v, Section 4.4) bounds the local
    error by (u_s + (n_d + n_q) u_q) sum_s |B_s| |r_s| plus the evaluation
    error of the FE functions; with u = 2^-24 and n_q = 512 the first factor
    is 3e-5, and cancellation in sum_s B_s r_s for rough (random) u costs a
    small further factor.
Degenerate input, unsupported forms and argument errors are checked too.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from fe_inputs import config_mesh, nodal_values, normal_vector
from paper_2410_12614_amd import _lib as L
from paper_2410_12614_amd import api

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()
    yield
    torch.cuda.synchronize()


def _kappa(x):
    return 1.0 + x[:, 0] * x[:, 1] + 0.5 * x[:, -1] ** 2


def _mesh(kind, n, p, flatten=0.05):
    if kind == "tri":
        return config_mesh("c1", n=n, degree=p)
    return config_mesh("c2", n=n, degree=p, flatten=flatten)


def _action(m, form, p, q, prec, coeff):
    desc = api.form_desc(m.d, p, q, form, prec, has_coeff=coeff is not None)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs, coeff)
    return api.Action(mv, desc)


def _dev(x, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.from_numpy(np.asarray(x)).to(dt).cuda().contiguous()


def _rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check(got, ref, prec, what):
    if prec == "fp64":
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"  {what}: max err {err:.2e}")
        assert err <= TOL["fp64"], what
    else:
        err = _rel2(got, ref)
        say(f"  {what}: rel 2-norm err {err:.2e}")
        assert err <= TOL["fp32"], what


CASES = [
    # kind, n, p, q, form, coefficient
    ("tet", 3, 1, 2, "stiffness", False),
    ("tet", 3, 2, 4, "mass", False),
    ("tet", 3, 2, 4, "stiffness", True),
    ("tet", 3, 3, 6, "mass", True),
    ("tet", 3, 4, 8, "stiffness", False),
    ("tet", 3, 4, 8, "mass", False),
    ("tet", 2, 5, 10, "stiffness", True),
    ("tet", 2, 6, 14, "stiffness", True),
    ("tet", 2, 6, 12, "mass", True),
    ("tri", 4, 2, 4, "stiffness", True),
    ("tri", 4, 5, 10, "mass", False),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}-p{c[2]}q{c[3]}-{c[4]}"
                         f"{'-z' if c[5] else ''}")
def test_action_and_vjp_match_oracle(case, prec):
    kind, n, p, q, form, with_z = case
    m = _mesh(kind, n, p)
    say(f"[action] {case} {prec}: {m.cell_coords.shape[0]} cells, {m.n_dofs} dofs")
    z = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, p, _kappa) if with_z else None
    u = normal_vector(m.n_dofs, 3).astype(np.float64)
    v = normal_vector(m.n_dofs, 4).astype(np.float64)
    act = _action(m, form, p, q, prec, z)
    y = act.apply(_dev(u, prec))
    gu, gz = act.vjp(_dev(u, prec), _dev(v, prec))
    torch.cuda.synchronize()
    assert api.fe_get_device_status(act.form_buf) == L.FE_OK
    y_ref = oracle.action(form, m, q, u, coeff=z)
    gu_ref, gz_ref = oracle.vjp(form, m, q, u, v, coeff=z)
    _check(y.double().cpu().numpy(), y_ref, prec, "y = A u")
    _check(gu.double().cpu().numpy(), gu_ref, prec, "grad_u = A^T v")
    if with_z:
        _check(gz.double().cpu().numpy(), gz_ref, prec, "grad_z")
    else:
        assert gz is None


def test_repeatable_and_ragged_batches():
    # 162 cells: ten full batches of 16 and a ragged batch of 2
    m = _mesh("tet", 3, 4)
    act = _action(m, "stiffness", 4, 8, "fp32", None)
    u = _dev(normal_vector(m.n_dofs, 3), "fp32")
    a = act.apply(u).clone()
    b = act.apply(u).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for n_cells in (1, 16, 17, 33):
        sub = type(m)(**{**m.__dict__, "cell_coords": m.cell_coords[:n_cells],
                         "dofmap": m.dofmap[:n_cells]})
        say(f"[action] ragged {n_cells} cells")
        act2 = _action(sub, "stiffness", 4, 8, "fp64", None)
        uu = normal_vector(m.n_dofs, 5).astype(np.float64)
        y = act2.apply(_dev(uu, "fp64")).cpu().numpy()
        ref = oracle.action("stiffness", sub, 8, uu)
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_empty_mesh_writes_zeros():
    m = _mesh("tet", 1, 2)
    sub = type(m)(**{**m.__dict__, "cell_coords": m.cell_coords[:0], "dofmap": m.dofmap[:0]})
    act = _action(sub, "mass", 2, 4, "fp32", None)
    y = torch.full((m.n_dofs,), 7.0, device="cuda")
    act.apply(_dev(np.ones(m.n_dofs), "fp32"), out=y)
    torch.cuda.synchronize()
    assert torch.count_nonzero(y).item() == 0


def test_degenerate_cell_reports_status():
    m = _mesh("tet", 2, 2, flatten=0.0)
    cc = m.cell_coords.copy()
    cc[3, 3] = cc[3, 0]                      # a vertex on top of another: det J = 0
    bad = type(m)(**{**m.__dict__, "cell_coords": cc})
    act = _action(bad, "stiffness", 2, 4, "fp64", None)
    y = act.apply(_dev(np.ones(m.n_dofs), "fp64"))
    torch.cuda.synchronize()
    assert api.fe_get_device_status(act.form_buf) == L.FE_EDEGENERATE
    assert torch.isnan(y).any()


def test_argument_errors():
    m = _mesh("tet", 1, 2)
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
    # unsupported precisions and degrees are refused before anything runs
    for prec, p in (("fp16", 2), ("fp32", 7)):
        desc = api.form_desc(3, p, 2 * p, "mass", prec)
        wb = ctypes.c_size_t(0)
        st = api.fe_action_vjp(desc, None, mv, None, L.FE_ACTION, None, None, None, None, None,
                               None, None, wb)
        assert st == L.FE_EUNSUPPORTED
    act = _action(m, "mass", 2, 4, "fp32", None)
    x = _dev(np.ones(m.n_dofs), "fp32")
    out = torch.empty_like(x)
    # a coefficient gradient without a coefficient
    st = api.fe_action_vjp(act.desc, act.form_buf, act.mesh, act.vplan, L.FE_VJP, x, x, None,
                           out, out, act.workspace)
    assert st == L.FE_EINVAL
    # a bad mode, a missing plan
    st = api.fe_action_vjp(act.desc, act.form_buf, act.mesh, act.vplan, 7, x, None, out, None,
                           None, act.workspace)
    assert st == L.FE_EINVAL
    st = api.fe_action_vjp(act.desc, act.form_buf, act.mesh, None, L.FE_ACTION, x, None, out,
                           None, None, act.workspace)
    assert st == L.FE_EINVAL
    # a plan of another mesh: detected on the device, nothing written
    m2 = _mesh("tet", 2, 2)
    act2 = _action(m2, "mass", 2, 4, "fp32", None)
    out.fill_(3.0)
    st = api.fe_action_vjp(act.desc, act.form_buf, act.mesh, act2.vplan, L.FE_ACTION, x, None,
                           out, None, None, act.workspace)
    assert st == L.FE_OK
    torch.cuda.synchronize()
    assert api.fe_get_device_status(act.form_buf) == L.FE_EINVAL
    assert bool((out == 3.0).all())


def test_autograd_function_matches_oracle_and_finite_differences():
    p, q = 3, 6
    m = _mesh("tet", 2, p)
    z = nodal_values(m.cell_coords, m.dofmap, m.n_dofs, p, _kappa)
    act = _action(m, "stiffness", p, q, "fp64", z)
    u0 = normal_vector(m.n_dofs, 3).astype(np.float64)
    v0 = normal_vector(m.n_dofs, 4).astype(np.float64)
    u = _dev(u0, "fp64").requires_grad_(True)
    coeff = act.mesh.coeff.requires_grad_(True)
    y = api.ActionFunction.apply(u, coeff, act)
    (y * _dev(v0, "fp64")).sum().backward()
    gu_ref, gz_ref = oracle.vjp("stiffness", m, q, u0, v0, coeff=z)
    gu, gz = u.grad.cpu().numpy(), coeff.grad.detach().cpu().numpy()
    assert np.abs(gu - gu_ref).max() <= 1e-12 * np.abs(gu_ref).max()
    assert np.abs(gz - gz_ref).max() <= 1e-12 * np.abs(gz_ref).max()
    # central differences of f(z) = v^T A(z) u through the GPU action (FP64,
    # h = 1e-6): f is linear in z, so only rounding separates the two
    coeff.requires_grad_(False)
    h = 1e-6
    vt = _dev(v0, "fp64")
    rng = np.random.default_rng(3)
    for dof in rng.choice(m.n_dofs, 8, replace=False):
        with torch.no_grad():
            coeff[dof] += h
            fp = float(vt @ act.apply(_dev(u0, "fp64")))
            coeff[dof] -= 2 * h
            fm = float(vt @ act.apply(_dev(u0, "fp64")))
            coeff[dof] += h
        fd = (fp - fm) / (2 * h)
        assert abs(fd - gz[dof]) <= 1e-5 * max(1.0, abs(gz[dof])), (dof, fd, gz[dof])


_FULL = {}


def _full_c5():
    if "mesh" not in _FULL:
        say("[action] building the full P6 mesh (196,608 cells)")
        m = config_mesh("c5")
        _FULL["mesh"] = m
        u = normal_vector(m.n_dofs, 3)
        v = normal_vector(m.n_dofs, 4)
        _FULL["u"], _FULL["v"] = u, v
        say("[action] oracle action and VJP at full size")
        _FULL["y"] = oracle.action("stiffness", m, 14, u.astype(np.float64), coeff=m.coeff)
        _FULL["gu"], _FULL["gz"] = oracle.vjp("stiffness", m, 14, u.astype(np.float64),
                                              v.astype(np.float64), coeff=m.coeff)
    return _FULL


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_size_weighted_p6_action_and_vjp(prec):
    F = _full_c5()
    m = F["mesh"]
    say(f"[action] full size P6 weighted stiffness {prec}")
    act = _action(m, "stiffness", 6, 14, prec, m.coeff)
    y = act.apply(_dev(F["u"], prec))
    gu, gz = act.vjp(_dev(F["u"], prec), _dev(F["v"], prec))
    torch.cuda.synchronize()
    assert api.fe_get_device_status(act.form_buf) == L.FE_OK
    _check(y.double().cpu().numpy(), F["y"], prec, "y")
    _check(gu.double().cpu().numpy(), F["gu"], prec, "grad_u")
    _check(gz.double().cpu().numpy(), F["gz"], prec, "grad_z")
