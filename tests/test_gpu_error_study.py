"""Rounding-error study of the mixed-precision kernels against degree (the
paper's study of Section 5.4, on the gfx950 path).

For every degree p = 1..8 (tetrahedra, quadrature degree 2p, 5 % of the
cells flattened to aspect 1e3) and both forms, the local matrices of each
GPU mode are compared with the FP64 oracle through the paper's normalised
error

    e = max_K ||A_K - Â_K||_max / (u_s ||A_K||_max),

u_s the storage unit roundoff of the mode (FP16 2^-11, BF16 2^-8, the
split pair 2^-22, FP32 2^-24).  Corollary 4.10 bounds it by
(1 + n_q u_q / u_s) kappa_q^A plus evaluation and geometry terms that are
negligible here (u_p, u_g <= FP32 / FP64), with
kappa_q^A = ||sum_st |B_s||H_st| ||_max / ||A||_max computed per cell below.
With FP32 accumulation (u_q = 2^-24) the FP16 and BF16 modes keep
n_q u_q / u_s < 0.1 up to n_q = 729, so their normalised errors are O(1)
times kappa_q^A and flat in p; a kernel run entirely in FP16 (geometry in
FP32, as in the paper's comparator; emulated here on the host with every
product and sum rounded to FP16) has u_q = u_s and its errors grow with n_q.
The measured table is printed (run with -s).
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

U_S = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "split": 2.0 ** -22, "fp32": 2.0 ** -24}
DEGREES = range(1, 9)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.load()
    yield
    torch.cuda.synchronize()


def _kappa_q(form, cells, tab):
    """kappa_q^A per cell (coefficient 1, positive weights)."""
    _, w, vals, grads = tab
    Bs = [vals] if form == "mass" else list(grads)            # [n_q][n_phi] each
    nd = len(Bs)
    Mabs = [[np.abs(Bs[s]).T @ (w[:, None] * np.abs(Bs[t])) for t in range(nd)]
            for s in range(nd)]
    out = []
    for x in cells:
        _, det, _, G = oracle.geometry(x)
        if form == "mass":
            G = np.array([[abs(det)]])
        S = sum(abs(G[s, t]) * Mabs[s][t] for s in range(nd) for t in range(nd))
        out.append(S)
    return out


def _fully_fp16(form, cells, tab):
    """Local matrices with every product and sum in FP16 (B, weights and the
    geometry tensor rounded to FP16; geometry computed in FP32), summed over
    the quadrature points in order."""
    h = np.float16
    _, w, vals, grads = tab
    Bs = [vals] if form == "mass" else list(grads)
    nd = len(Bs)
    Bh = [b.astype(h) for b in Bs]
    wh = w.astype(h)
    res = []
    for x in cells:
        x32 = x.astype(np.float32)
        J = (x32[1:] - x32[0]).T
        det = np.float32(np.linalg.det(J))
        Ji = np.linalg.inv(J).astype(np.float32)
        G = (abs(det) * (Ji @ Ji.T)).astype(np.float32) if form == "stiffness" \
            else np.array([[abs(det)]], np.float32)
        Gh = G.astype(h)
        A = np.zeros((Bs[0].shape[1],) * 2, dtype=h)
        for s in range(nd):
            for t in range(nd):
                for q in range(len(w)):
                    c = h(wh[q] * Gh[s, t])
                    Hq = (c * Bh[t][q]).astype(h)                     # H_st row q
                    A = (A + np.outer(Bh[s][q], Hq).astype(h)).astype(h)
        res.append(A.astype(np.float64))
    return res


def _normalised(A_ref, A_got, u_s):
    return max(np.abs(a - b).max() / (u_s * np.abs(a).max()) for a, b in zip(A_ref, A_got))


_RESULTS = {}


@pytest.mark.parametrize("form", ["mass", "stiffness"])
def test_mixed_precision_errors_are_flat_in_degree(form):
    rows = []
    for p in DEGREES:
        q = 2 * p
        m = config_mesh("c2", n=2, degree=p, flatten=0.05)
        tab = oracle.tabulation(3, p, q)
        ref = oracle.local_matrices(form, m.cell_coords, p, q, tab=tab)
        kap = max(S.max() / np.abs(A).max() for S, A in zip(_kappa_q(form, m.cell_coords, tab), ref))
        n_q = len(tab[1])
        row = {"p": p, "n_q": n_q, "kappa_q": kap}
        mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
        for prec in ("fp16", "bf16", "split", "fp32"):
            desc = api.form_desc(3, p, q, form, prec)
            buf = api.fe_form_prepare(desc)
            out = torch.empty((m.cell_coords.shape[0], m.n_phi, m.n_phi), device="cuda")
            api.fe_cell_kernels(desc, buf, mv, out)
            torch.cuda.synchronize()
            assert api.fe_get_device_status(buf) == L.FE_OK
            row[prec] = _normalised(ref, out.double().cpu().numpy(), U_S[prec])
        # the fully-FP16 comparator on the first cells (host emulation)
        nc = (1 if form == "stiffness" else 2) if p >= 7 else 4
        row["full_fp16"] = _normalised(ref[:nc], _fully_fp16(form, m.cell_coords[:nc], tab),
                                       U_S["fp16"])
        rows.append(row)
        say(f"  {form} p={p} n_q={n_q:4d} kappa_q={kap:7.2f}  " +
            "  ".join(f"{k}={row[k]:8.3f}" for k in ("fp16", "bf16", "split", "fp32", "full_fp16")))
    _RESULTS[form] = rows
    for r in rows:
        # Corollary 4.10 with u_q = 2^-24: O(1) kappa_q^A, a few roundings of
        # the stored factors (B, w B, G, H in FP16) per term
        assert r["fp16"] <= 8 * r["kappa_q"], r
        assert r["bf16"] <= 4 * r["kappa_q"], r
    for mode in ("fp16", "bf16"):
        v = [r[mode] for r in rows]
        assert max(v) <= 10 * min(v), (mode, v)       # flat in p
    # the FP16 accumulation of the fully-FP16 kernel makes its error grow with n_q
    assert rows[-1]["full_fp16"] > 2 * rows[0]["full_fp16"], [r["full_fp16"] for r in rows]
