"""FP64 CPU oracle for the cell kernels and global CSR assembly.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library neither imports it nor shares code, headers, tables or helpers with
it; both sides receive the same seeded inputs from ``fe_inputs``.

Parts and what pins them (tests under ``tests/test_oracle_*.py``):

* ``quadrature``: collapsed Gauss-Jacobi rules (Golub-Welsch) -- pinned by
  exact rational monomial integrals, by ``scipy.special.roots_jacobi`` and by
  50-digit ``mpmath`` Gauss-Jacobi nodes.
* ``basis``: Silvester product-form Lagrange basis (Appendix A) -- pinned by
  the Kronecker property, partition of unity, linear reproduction, the
  dimension formula and P1 = barycentric coordinates.
* ``oracle_fe.c`` geometry (Section 4.2) -- pinned by the paper's
  epsilon-tetrahedron (det J = eps, kappa_inf closed form), rigid-motion
  invariance, dilation scaling and ``numpy.linalg``.
* ``oracle_fe.c`` local matrices (Algorithm 1) -- pinned by P1 closed forms,
  the mass identity A_K = |det J| M_ref, the reference-tensor route, symmetry
  and zero row sums.
* ``oracle_fe.c`` assembly (Section 3.3) -- pinned by brute-force dense
  assembly on tiny meshes, nnz counts, and exact polynomial integrals
  u^T M v, u^T K v.
* ``hexahedra.py`` (rule and Q_p basis) with ``oracle_fe.c``'s
  ``oracle_hex_local_matrices`` (boxed cells, geometry tensor per
  quadrature point of the trilinear map): mass and stiffness matrices --
  pinned by exact monomial integrals of the tensor rule, the Kronecker
  property, the unit cube = Kronecker sums and products of exact rational 1D
  mass and stiffness matrices, the volume of a jittered mesh, zero row sums
  of the stiffness matrix, x^T K x = |Omega| for the coordinate function
  (which lies in Q_1 on a trilinear cell), and exact polynomial integrals.
* ``oracle_fe.c`` actions (Algorithm 2) and the coefficient adjoint -- pinned
  by the assembled matrix times the vector (Algorithm 1 route), mass and
  stiffness actions on constants (|Omega|, zero), the exact integral of
  w grad u . grad v for polynomials, the Euler identity
  sum_m z_m g_m = v^T A(z) u, brute force g_m = v^T A(e_m) u, and central
  finite differences of the patch functional.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from . import basis, quadrature  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_fe.c")
_LIB = os.path.join(_HERE, "liboracle_fe.so")

FORM_MASS = 0
FORM_STIFFNESS = 1
FORMS = {"mass": FORM_MASS, "stiffness": FORM_STIFFNESS}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C part with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_geometry.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.oracle_geometry.restype = ctypes.c_int
        lib.oracle_local_matrices.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P,
                                              ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                              ctypes.c_int]
        lib.oracle_local_matrices.restype = ctypes.c_int
        lib.oracle_csr_pattern.argtypes = [ctypes.c_int64, ctypes.c_int, P, ctypes.c_int64, P, P]
        lib.oracle_csr_pattern.restype = ctypes.c_int64
        lib.oracle_assemble.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, ctypes.c_int64, P,
                                        P, P]
        lib.oracle_assemble.restype = ctypes.c_int
        lib.oracle_local_vectors.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P,
                                             ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P,
                                             P, P, ctypes.c_int]
        lib.oracle_local_vectors.restype = ctypes.c_int
        lib.oracle_assemble_vector.argtypes = [ctypes.c_int64, ctypes.c_int, P, P,
                                               ctypes.c_int64, P]
        lib.oracle_assemble_vector.restype = ctypes.c_int
        lib.oracle_hex_local_matrices.argtypes = [ctypes.c_int, ctypes.c_int64, P, ctypes.c_int,
                                                  ctypes.c_int, P, P, P, P, P, ctypes.c_int]
        lib.oracle_hex_local_matrices.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def geometry(x: np.ndarray):
    """(J, det J, J^{-1}, G_poisson) of one simplex with vertices x [d+1][d]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    d = x.shape[1]
    J = np.zeros((d, d)); Ji = np.zeros((d, d)); G = np.zeros((d, d))
    det = np.zeros(1)
    st = _load().oracle_geometry(d, _ptr(x), _ptr(J), _ptr(det), _ptr(Ji), _ptr(G))
    if st != 0:
        raise OracleError(f"degenerate cell (status {st})")
    return J, float(det[0]), Ji, G


def tabulation(d: int, degree: int, quad_degree: int):
    """(points, weights, values [n_q][n_phi], gradients [d][n_q][n_phi])."""
    pts, w = quadrature.collapsed_rule(d, quad_degree)
    vals, grads = basis.tabulate(d, degree, pts)
    return pts, w, vals, grads


def local_matrices(form: str, cell_coords: np.ndarray, degree: int, quad_degree: int,
                   dofmap: Optional[np.ndarray] = None, coeff: Optional[np.ndarray] = None,
                   nthreads: int = 0, tab=None) -> np.ndarray:
    """Element matrices A_K [n_cells][n_phi][n_phi] by Algorithm 1 in FP64."""
    cc = np.ascontiguousarray(cell_coords, dtype=np.float64)
    n_cells, dp1, d = cc.shape
    if tab is None:
        tab = tabulation(d, degree, quad_degree)
    _, w, vals, grads = tab
    w = np.ascontiguousarray(w); vals = np.ascontiguousarray(vals)
    grads = np.ascontiguousarray(grads)
    n_q, n_phi = vals.shape
    A = np.empty((n_cells, n_phi, n_phi))
    dm = None if dofmap is None else np.ascontiguousarray(dofmap, dtype=np.int32)
    cf = None if coeff is None else np.ascontiguousarray(coeff, dtype=np.float64)
    st = _load().oracle_local_matrices(d, FORMS[form], n_cells, _ptr(cc), n_phi, n_q, _ptr(w),
                                       _ptr(vals), _ptr(grads), _ptr(dm), _ptr(cf), _ptr(A),
                                       int(nthreads))
    if st != 0:
        raise OracleError(f"oracle_local_matrices failed (status {st})")
    return A


def csr_pattern(dofmap: np.ndarray, n_dofs: int):
    """(row_ptr int64 [n_dofs+1], col_idx int32 [nnz])."""
    dm = np.ascontiguousarray(dofmap, dtype=np.int32)
    n_cells, n_phi = dm.shape
    row_ptr = np.zeros(n_dofs + 1, dtype=np.int64)
    lib = _load()
    nnz = lib.oracle_csr_pattern(n_cells, n_phi, _ptr(dm), n_dofs, _ptr(row_ptr), None)
    if nnz < 0:
        raise OracleError(f"oracle_csr_pattern failed ({nnz})")
    col = np.zeros(nnz, dtype=np.int32)
    nnz2 = lib.oracle_csr_pattern(n_cells, n_phi, _ptr(dm), n_dofs, _ptr(row_ptr), _ptr(col))
    assert nnz2 == nnz
    return row_ptr, col


def assemble(dofmap: np.ndarray, A_local: np.ndarray, n_dofs: int, row_ptr=None, col_idx=None):
    """CSR (row_ptr, col_idx, values) of L D L^T in FP64."""
    dm = np.ascontiguousarray(dofmap, dtype=np.int32)
    if row_ptr is None:
        row_ptr, col_idx = csr_pattern(dm, n_dofs)
    Al = np.ascontiguousarray(A_local, dtype=np.float64)
    vals = np.zeros(int(row_ptr[-1]))
    st = _load().oracle_assemble(dm.shape[0], dm.shape[1], _ptr(dm), _ptr(Al), n_dofs,
                                 _ptr(row_ptr), _ptr(col_idx), _ptr(vals))
    if st != 0:
        raise OracleError(f"oracle_assemble failed ({st})")
    return row_ptr, col_idx, vals


def assemble_form(form: str, mesh, quad_degree: int, nthreads: int = 0, coeff=None):
    """Convenience: local matrices of ``form`` on ``mesh`` then CSR assembly."""
    A = local_matrices(form, mesh.cell_coords, mesh.degree, quad_degree, mesh.dofmap,
                       coeff, nthreads)
    return assemble(mesh.dofmap, A, mesh.n_dofs)


def local_vectors(form: str, cell_coords: np.ndarray, degree: int, quad_degree: int,
                  dofmap: np.ndarray, u: np.ndarray, coeff: Optional[np.ndarray] = None,
                  v: Optional[np.ndarray] = None, nthreads: int = 0, tab=None):
    """(b, g): local action vectors b_K by Algorithm 2 for the FE function u,
    [n_cells][n_phi], and, when ``v`` is given, the local coefficient adjoint
    g_K of f(z) = v^T A(z) u (else None), all in FP64."""
    cc = np.ascontiguousarray(cell_coords, dtype=np.float64)
    n_cells, _, d = cc.shape
    if tab is None:
        tab = tabulation(d, degree, quad_degree)
    _, w, vals, grads = tab
    w = np.ascontiguousarray(w); vals = np.ascontiguousarray(vals)
    grads = np.ascontiguousarray(grads)
    n_q, n_phi = vals.shape
    dm = np.ascontiguousarray(dofmap, dtype=np.int32)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    cf = None if coeff is None else np.ascontiguousarray(coeff, dtype=np.float64)
    b = np.empty((n_cells, n_phi))
    g = None if v is None else np.empty((n_cells, n_phi))
    st = _load().oracle_local_vectors(d, FORMS[form], n_cells, _ptr(cc), n_phi, n_q, _ptr(w),
                                      _ptr(vals), _ptr(grads), _ptr(dm), _ptr(cf), _ptr(uu),
                                      _ptr(vv), _ptr(b), _ptr(g), int(nthreads))
    if st != 0:
        raise OracleError(f"oracle_local_vectors failed (status {st})")
    return b, g


def assemble_vector(dofmap: np.ndarray, b: np.ndarray, n_dofs: int) -> np.ndarray:
    """v^g = L b in FP64, summed in the order cell ascending, then i."""
    dm = np.ascontiguousarray(dofmap, dtype=np.int32)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    out = np.empty(n_dofs)
    st = _load().oracle_assemble_vector(dm.shape[0], dm.shape[1], _ptr(dm), _ptr(bb), n_dofs,
                                        _ptr(out))
    if st != 0:
        raise OracleError(f"oracle_assemble_vector failed ({st})")
    return out


def action(form: str, mesh, quad_degree: int, u: np.ndarray, coeff=None, nthreads: int = 0):
    """y = A(z) u by Algorithm 2 on every cell, then vector assembly."""
    b, _ = local_vectors(form, mesh.cell_coords, mesh.degree, quad_degree, mesh.dofmap, u,
                         coeff, None, nthreads)
    return assemble_vector(mesh.dofmap, b, mesh.n_dofs)


def vjp(form: str, mesh, quad_degree: int, u: np.ndarray, v: np.ndarray, coeff=None,
        nthreads: int = 0):
    """Cotangent v of y = A(z) u: (grad_u, grad_z) with grad_u = A(z)^T v
    (= A(z) v: both forms are symmetric) and grad_z[m] = v^T (dA/dz_m) u
    (None without a coefficient)."""
    b, g = local_vectors(form, mesh.cell_coords, mesh.degree, quad_degree, mesh.dofmap, v,
                         coeff, u if coeff is not None else None, nthreads)
    gu = assemble_vector(mesh.dofmap, b, mesh.n_dofs)
    gz = None if g is None else assemble_vector(mesh.dofmap, g, mesh.n_dofs)
    return gu, gz
