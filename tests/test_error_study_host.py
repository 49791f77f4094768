"""Rounding-error experiments of Sections 5.2 and 5.3 that need arithmetic
the matrix cores do not offer (FP16 accumulation, FP16 geometry): emulated
on the host with every operation rounded to the stated format, against the
FP64 oracle.  Run with -s to print the tables.

Section 5.3 (accumulation of matrix-matrix products).  Mass bilinear form
and mass action on tetrahedra, single precision for storage, geometry and
FE function evaluation (u_s = u_g = u_p = 2^-24) and half precision for the
products and their accumulation (u_q = 2^-11), so that the O(u_q) term of
the local-kernel error theorem dominates.  The paper monitors

    max_K ||A_K - Â_K||_max / (u_q ||A_K||_max)    (bilinear form)
    max_K ||v_K - v̂_K||_inf / (u_q ||v_K||_inf)    (action)

against n_q: the worst-case bound grows like n_q, independent random
rounding errors would give n_q^(1/2), and the paper observes a rate close to
1 for actions and about 0.7 for bilinear forms (cell by cell between 0.5
and 1).  Here the rate is the least-squares slope of log(error) against
log(n_q) over p = 2..8 (the paper's degrees start at 2; quadrature degree
2p, n_q = (p+1)^3), the maximum taken over 24 cells of a jittered mesh.
The action is applied to the FE function with every dof equal to 1 (the
paper fixes the coefficient to 1 and does not state the function).

Section 5.2 (geometry).  The paper's epsilon-tetrahedron (scaled by 3^-1/2
and translated, so that the coordinates are not exact), Poisson geometry
G = |det J| J^-1 J^-T by the cofactor formula, every operation rounded to
single or to half: the single-precision error grows linearly with
kappa_2(J) with a constant around 0.1, and half precision loses every digit
at condition numbers of about 10^4.5 (the paper predicts this and reports
that its half computation underflows: det J leaves the normal half range).
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from fe_inputs import config_mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eps_tetrahedron.json")
U16 = 2.0 ** -11
U32 = 2.0 ** -24


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def fl16(x):
    """Round to half (round to nearest even), returned as float64: products
    of singles and sums of halves are exact in double, so rounding the exact
    double result once is the correctly rounded half operation."""
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def fl32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def det32(x):
    """|det J| of a tetrahedron, coordinates and every operation in single
    (cofactor expansion)."""
    x = x.astype(np.float32)
    J = (x[1:] - x[0]).T
    a = J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1]
    b = J[1, 0] * J[2, 2] - J[1, 2] * J[2, 0]
    c = J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]
    return float(np.float32(abs(J[0, 0] * a - J[0, 1] * b + J[0, 2] * c)))


def _pow2_scale(m):
    """Exact power of two that brings m into [2^8, 2^9) (keeps half sums in range)."""
    return 2.0 ** (8 - int(np.floor(np.log2(m))))


def _mass_bilinear_fp16acc(x, tab):
    """Mass matrix with single storage/geometry and half products and sums,
    accumulated over the quadrature points in order."""
    _, w, vals, _ = tab
    B = fl32(vals)
    c = fl32(fl32(w) * det32(x))
    H = fl32(c[:, None] * B)                                   # [q][j], u_s = single
    sig = _pow2_scale((np.abs(B).T @ np.abs(H)).max())
    Hs = H * sig                                               # exact
    S = np.zeros((B.shape[1], B.shape[1]))
    for q in range(len(w)):
        S = fl16(S + fl16(np.outer(B[q], Hs[q])))
    return S / sig


def _mass_action_fp16acc(x, tab, u):
    """Mass action v_i = sum_q B(q, i) r_q, r_q = c_q u_h(X_q): u_h evaluated
    in single, products and sums over q in half."""
    _, w, vals, _ = tab
    B = fl32(vals)
    c = fl32(fl32(w) * det32(x))
    uq = (B.astype(np.float32) @ u.astype(np.float32)).astype(np.float64)   # u_p = single
    r = fl32(c * uq)
    sig = _pow2_scale((np.abs(B).T @ np.abs(r)).max())
    rs = r * sig
    v = np.zeros(B.shape[1])
    for q in range(len(w)):
        v = fl16(v + fl16(B[q] * rs[q]))
    return v / sig


def _rate(n_q, err):
    return float(np.polyfit(np.log(n_q), np.log(err), 1)[0])


@pytest.fixture(scope="module")
def accumulation_table():
    rows = []
    for p in range(2, 9):
        q = 2 * p
        m = config_mesh("c2", n=2, degree=p, flatten=0.0)
        cells = m.cell_coords[:24]
        tab = oracle.tabulation(3, p, q)
        n_q = len(tab[1])
        A = oracle.local_matrices("mass", cells, p, q, tab=tab)
        dm = np.arange(len(cells) * m.n_phi, dtype=np.int32).reshape(len(cells), m.n_phi)
        u = np.ones(dm.size)
        b, _ = oracle.local_vectors("mass", cells, p, q, dm, u, tab=tab)
        eA = [np.abs(A[k] - _mass_bilinear_fp16acc(cells[k], tab)).max() / (U16 * np.abs(A[k]).max())
              for k in range(len(cells))]
        ev = [np.abs(b[k] - _mass_action_fp16acc(cells[k], tab, u[dm[k]])).max() /
              (U16 * np.abs(b[k]).max()) for k in range(len(cells))]
        rows.append({"p": p, "n_q": n_q, "bilinear": max(eA), "action": max(ev),
                     "bilinear_cells": eA, "action_cells": ev})
        say(f"  p={p} n_q={n_q:4d}  bilinear {max(eA):8.3f}  action {max(ev):8.3f}")
    return rows


def test_fp16_accumulation_error_grows_with_n_q(accumulation_table):
    rows = accumulation_table
    n_q = np.array([r["n_q"] for r in rows], dtype=float)
    rb = _rate(n_q, [r["bilinear"] for r in rows])
    ra = _rate(n_q, [r["action"] for r in rows])
    per_cell = [_rate(n_q, [r["bilinear_cells"][k] for r in rows])
                for k in range(len(rows[0]["bilinear_cells"]))]
    say(f"  fitted rate in n_q: bilinear {rb:.2f}, action {ra:.2f}; "
        f"per-cell bilinear rates {min(per_cell):.2f} .. {max(per_cell):.2f}")
    # the paper: actions close to 1, bilinear forms about 0.7, cells between
    # 0.5 and 1; the worst-case bound is rate 1 (n_q u_q)
    assert 0.5 <= rb <= 1.0, rb
    assert 0.5 <= ra <= 1.0, ra
    # errors stay within the worst-case constant of the accumulation bound
    for r in rows:
        assert r["bilinear"] <= 2 * r["n_q"] and r["action"] <= 2 * r["n_q"], r


def eps_tet(eps):
    g = json.load(open(GOLDEN))["transform"]
    x = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [eps, 1, -1]], dtype=float)
    return x * 3 ** -0.5 + np.array(g["translate"])


def poisson_geometry(x, dtype):
    """G = |det J| J^-1 J^-T = adj(J) adj(J)^T / |det J| with the coordinates
    and every operation rounded to ``dtype`` (numpy rounds each half or
    single operation correctly)."""
    x = x.astype(dtype)
    J = (x[1:] - x[0]).T
    adj = np.empty((3, 3), dtype=dtype)
    adj[0, 0] = J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1]
    adj[0, 1] = J[0, 2] * J[2, 1] - J[0, 1] * J[2, 2]
    adj[0, 2] = J[0, 1] * J[1, 2] - J[0, 2] * J[1, 1]
    adj[1, 0] = J[1, 2] * J[2, 0] - J[1, 0] * J[2, 2]
    adj[1, 1] = J[0, 0] * J[2, 2] - J[0, 2] * J[2, 0]
    adj[1, 2] = J[0, 2] * J[1, 0] - J[0, 0] * J[1, 2]
    adj[2, 0] = J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]
    adj[2, 1] = J[0, 1] * J[2, 0] - J[0, 0] * J[2, 1]
    adj[2, 2] = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
    det = J[0, 0] * adj[0, 0] + J[0, 1] * adj[1, 0] + J[0, 2] * adj[2, 0]
    G = np.empty((3, 3), dtype=dtype)
    with np.errstate(all="ignore"):
        for i in range(3):
            for j in range(3):
                s = adj[i, 0] * adj[j, 0]
                s = s + adj[i, 1] * adj[j, 1]
                s = s + adj[i, 2] * adj[j, 2]
                G[i, j] = s / abs(det)
    return G.astype(np.float64), float(det)


def test_geometry_precision_sweep():
    rows = []
    for e in range(1, 11):
        eps = 10.0 ** -e
        x = eps_tet(eps)
        J, det, _, G = oracle.geometry(x)
        k2 = np.linalg.cond(J, 2)
        r = {"eps": eps, "kappa2": k2}
        for name, dt, u in (("fp32", np.float32, U32), ("fp16", np.float16, U16)):
            Gh, dh = poisson_geometry(x, dt)
            err = np.abs(G - Gh).max() / (u * np.abs(G).max())
            r[name] = err if np.isfinite(err) else np.inf
            r[name + "_rel"] = r[name] * u
            r[name + "_det_subnormal"] = name == "fp16" and abs(dh) < 2.0 ** -14
        rows.append(r)
        say(f"  eps=1e-{e:<2d} kappa2={k2:9.3e}  fp32 {r['fp32']:9.3e} u  fp16 {r['fp16']:9.3e} u"
            f"{'  (det J subnormal in half)' if r['fp16_det_subnormal'] else ''}")
    # single: linear in kappa_2 with a constant of order 0.1 (slope 1 fitted
    # where the relative error is below 0.1), every digit kept up to
    # kappa_2 ~ 10^6 and lost only near 1/u_32 (the paper: safe to ~10^8.5)
    lin = [r for r in rows if r["fp32_rel"] < 0.1]
    k = np.array([r["kappa2"] for r in lin])
    e32 = np.array([r["fp32"] for r in lin])
    slope = np.polyfit(np.log(k), np.log(e32), 1)[0]
    say(f"  single precision: slope {slope:.2f} in kappa_2 (kappa_2 <= {k.max():.1e}), "
        f"error / kappa_2 between {(e32 / k).min():.3f} and {(e32 / k).max():.3f} u")
    assert len(lin) >= 5 and 0.8 <= slope <= 1.2, (len(lin), slope)
    assert (e32 <= 0.5 * k).all()
    assert all(r["fp32_rel"] < 0.1 for r in rows if r["kappa2"] <= 1e6)
    # half: every digit is lost (relative error >= 1/2, or no finite value)
    # once kappa_2 exceeds about 10^4 (the paper predicts 10^4.5): det J is a
    # cancellation of O(1) terms down to 0.19 eps, which half cannot resolve
    # (it comes out zero or subnormal)
    first = next(r for r in rows if r["fp16_rel"] >= 0.5)
    say(f"  half precision: every digit lost from kappa_2 = {first['kappa2']:.1e} on")
    assert first["kappa2"] <= 10 ** 5, first
    assert all(r["fp16_rel"] >= 0.5 for r in rows if r["kappa2"] >= first["kappa2"])
    assert first["fp16_det_subnormal"] or not np.isfinite(first["fp16"])
    # and it is still accurate to a few digits where the cell is well shaped
    assert rows[0]["fp16_rel"] <= 0.05, rows[0]
