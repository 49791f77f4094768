"""Thin Python binding of the C ABI (argument marshalling only).

Every function here forwards to ``libfe.so`` with the same name.  PyTorch
provides device memory and the HIP stream; no step of the computation runs
in Python.  ``Assembly`` is a convenience that allocates the caller-owned
buffers the ABI asks for and issues the phases in order.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import check

PRECISIONS = {
    "fp64": L.FE_FP64,
    "fp32": L.FE_FP32,
    "fp16": L.FE_FP16_ACC32,
    "bf16": L.FE_BF16_ACC32,
    "split": L.FE_SPLITFP16_ACC32,
}
FORMS = {"mass": L.FE_MASS, "stiffness": L.FE_STIFFNESS}


GEOMETRY = {"fp64": L.FE_GEOM_FP64, "fp32": L.FE_GEOM_FP32, "auto": L.FE_GEOM_AUTO}


def form_desc(d: int, degree: int, quad_degree: int, form: str, precision: str = "fp64",
              has_coeff: bool = False, geometry: str = "fp64") -> L.fe_form_desc:
    return L.fe_form_desc(cell=d, degree=degree, quad_degree=quad_degree, form=FORMS[form],
                          has_coeff=int(bool(has_coeff)), precision=PRECISIONS[precision],
                          geom_precision=GEOMETRY[geometry])


def _stream(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def fe_tabulate(cell: int, degree: int, quad_degree: int, nderiv: int = 1):
    """(points [n_q][d], weights [n_q], table [1 + d*nderiv][n_q][n_phi]) in FP64 (host);
    ``cell`` is FE_TRIANGLE (2), FE_TETRAHEDRON (3) or FE_HEXAHEDRON (8, d = 3)."""
    lib = L.load()
    d = 3 if cell == L.FE_HEXAHEDRON else cell
    n_phi, n_q = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib.fe_tabulate(cell, degree, quad_degree, nderiv, ctypes.byref(n_phi), ctypes.byref(n_q),
                          None, None, None), "fe_tabulate")
    pts = np.zeros((n_q.value, d))
    w = np.zeros(n_q.value)
    tab = np.zeros((1 + d * nderiv, n_q.value, n_phi.value))
    check(lib.fe_tabulate(cell, degree, quad_degree, nderiv, ctypes.byref(n_phi), ctypes.byref(n_q),
                          pts.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                          tab.ctypes.data_as(ctypes.c_void_p)), "fe_tabulate")
    return pts, w, tab


def fe_form_prepare(desc: L.fe_form_desc, device="cuda", stream=None) -> torch.Tensor:
    lib = L.load()
    size = ctypes.c_size_t(0)
    check(lib.fe_form_prepare(ctypes.byref(desc), None, ctypes.byref(size), None), "fe_form_prepare")
    buf = torch.empty(size.value, dtype=torch.uint8, device=device)
    check(lib.fe_form_prepare(ctypes.byref(desc), _ptr(buf), ctypes.byref(size), _stream(stream)),
          "fe_form_prepare")
    return buf


@dataclass
class MeshView:
    """Device views of a mesh: coords [n_cells][d+1][d] f64, dofmap [n_cells][n_phi] i32."""

    coords: torch.Tensor
    dofmap: torch.Tensor
    n_dofs: int
    coeff: Optional[torch.Tensor] = None

    @classmethod
    def from_numpy(cls, coords, dofmap, n_dofs, coeff=None, device="cuda") -> "MeshView":
        c = torch.from_numpy(np.ascontiguousarray(coords, dtype=np.float64)).to(device)
        m = torch.from_numpy(np.ascontiguousarray(dofmap, dtype=np.int32)).to(device)
        z = None if coeff is None else torch.from_numpy(np.ascontiguousarray(coeff, dtype=np.float64)).to(device)
        return cls(c, m, int(n_dofs), z)

    def struct(self) -> L.fe_mesh_view:
        for t, dt in ((self.coords, torch.float64), (self.dofmap, torch.int32)):
            if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("mesh tensors must be contiguous device tensors (f64 coords, i32 dofmap)")
        if self.coeff is not None and (self.coeff.dtype != torch.float64 or not self.coeff.is_contiguous()):
            raise ValueError("coeff must be a contiguous f64 device tensor")
        return L.fe_mesh_view(n_cells=self.coords.shape[0], cell_coords=self.coords.data_ptr(),
                              dofmap=self.dofmap.data_ptr(), n_dofs=self.n_dofs,
                              coeff=None if self.coeff is None else self.coeff.data_ptr())

    @property
    def n_cells(self) -> int:
        return int(self.coords.shape[0])


def fe_cell_kernels(desc: L.fe_form_desc, form_buf: torch.Tensor, mesh: MeshView,
                    A_local: torch.Tensor, stream=None) -> None:
    mv = mesh.struct()
    check(L.load().fe_cell_kernels(ctypes.byref(desc), _ptr(form_buf), ctypes.byref(mv),
                                   _ptr(A_local), _stream(stream)), "fe_cell_kernels")


def fe_get_device_status(buf: torch.Tensor, stream=None) -> int:
    return int(L.load().fe_get_device_status(_ptr(buf), _stream(stream)))


def fe_assemble_csr(descs: Sequence[L.fe_form_desc], form_bufs: Sequence[Optional[torch.Tensor]],
                    mesh: MeshView, phase: int, mats: "ctypes.Array", plan: Optional[torch.Tensor],
                    workspace: Optional[torch.Tensor], stream=None,
                    plan_bytes: Optional[ctypes.c_size_t] = None,
                    ws_bytes: Optional[ctypes.c_size_t] = None) -> int:
    n = len(descs)
    darr = (L.fe_form_desc * n)(*descs)
    barr = (ctypes.c_void_p * n)(*[None if b is None else b.data_ptr() for b in form_bufs])
    mv = mesh.struct()
    pb = plan_bytes if plan_bytes is not None else ctypes.c_size_t(0 if plan is None else plan.numel())
    wb = ws_bytes if ws_bytes is not None else ctypes.c_size_t(0 if workspace is None else workspace.numel())
    st = L.load().fe_assemble_csr(darr, barr, n, ctypes.byref(mv), phase, mats, _ptr(plan),
                                  ctypes.byref(pb), _ptr(workspace), ctypes.byref(wb), _stream(stream))
    return st


class Assembly:
    """Caller-side orchestration: sizes and allocates the buffers of the ABI
    (form buffers, plan, CSR arrays, workspace) with torch, then runs the
    symbolic phases once and the numeric phase on demand."""

    def __init__(self, mesh: MeshView, descs: Sequence[L.fe_form_desc], stream=None):
        self.mesh = mesh
        self.descs = list(descs)
        self.stream = stream
        dev = mesh.coords.device
        self.form_bufs = [fe_form_prepare(d, dev, stream) for d in self.descs]
        n = len(self.descs)
        self.mats = (L.fe_csr * n)()
        pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(fe_assemble_csr(self.descs, [None] * n, mesh, L.FE_NUMERIC, self.mats, None, None,
                              stream, pb, wb), "fe_assemble_csr(size query)")
        self.plan = torch.empty(pb.value, dtype=torch.uint8, device=dev)
        self.workspace = torch.empty(wb.value, dtype=torch.uint8, device=dev)
        self.row_ptr = torch.empty(mesh.n_dofs + 1, dtype=torch.int64, device=dev)
        for k in range(n):
            self.mats[k].n_rows = mesh.n_dofs
            self.mats[k].row_ptr = self.row_ptr.data_ptr()
        check(fe_assemble_csr(self.descs, self.form_bufs, mesh, L.FE_SYMBOLIC_COUNT, self.mats,
                              self.plan, None, stream), "fe_assemble_csr(COUNT)")
        self.nnz = int(self.mats[0].nnz)
        self.col_idx = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        vdt = torch.float64 if self.descs[0].precision == L.FE_FP64 else torch.float32
        self.values = [torch.empty(max(self.nnz, 1), dtype=vdt, device=dev) for _ in range(n)]
        for k in range(n):
            self.mats[k].col_idx = self.col_idx.data_ptr()
            self.mats[k].values = self.values[k].data_ptr()
        check(fe_assemble_csr(self.descs, self.form_bufs, mesh, L.FE_SYMBOLIC_FILL, self.mats,
                              self.plan, None, stream), "fe_assemble_csr(FILL)")
        self.graph = None

    def numeric(self, gather: bool = False, part: Optional[str] = None) -> list:
        """FE_NUMERIC (fused row-ownership path where it applies) or, with
        ``gather``, FE_NUMERIC_GATHER (cell kernels + row gather); ``part``
        "geometry" or "fused" runs one half of the fused FE_NUMERIC, "local"
        or "assemble" one half of FE_NUMERIC_GATHER."""
        phase = L.FE_NUMERIC_GATHER if gather else L.FE_NUMERIC
        if part is not None:
            phase = {"geometry": L.FE_NUMERIC_GEOMETRY, "fused": L.FE_NUMERIC_FUSED,
                     "local": L.FE_NUMERIC_LOCAL, "assemble": L.FE_NUMERIC_ASSEMBLE}[part]
        check(fe_assemble_csr(self.descs, self.form_bufs, self.mesh, phase, self.mats,
                              self.plan, self.workspace, self.stream), "fe_assemble_csr(NUMERIC)")
        return self.values

    def capture(self, gather: bool = False, part: Optional[str] = None) -> None:
        """Record numeric(gather, part) as one HIP graph (the numeric phases
        launch kernels only: no copies, fills or synchronisations), which
        replay() then runs; on torch's current stream, so the assembly's
        own stream must be the default (None)."""
        if self.stream is not None:
            raise ValueError("capture() records on torch's current stream; the assembly has its own")
        self.numeric(gather, part)           # first launches outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.numeric(gather, part)
        self.graph = g

    def replay(self) -> list:
        if self.graph is None:
            raise RuntimeError("replay() before capture()")
        self.graph.replay()
        return self.values

    def numeric_noalloc(self) -> list:
        """FE_NUMERIC through fe_assemble_csr_noalloc: the fused path with the
        library's own scratch array instead of ``self.workspace``."""
        n = len(self.descs)
        darr = (L.fe_form_desc * n)(*self.descs)
        barr = (ctypes.c_void_p * n)(*[b.data_ptr() for b in self.form_bufs])
        mv = self.mesh.struct()
        check(L.load().fe_assemble_csr_noalloc(darr, barr, n, ctypes.byref(mv), self.mats,
                                               _ptr(self.plan), _stream(self.stream)),
              "fe_assemble_csr_noalloc")
        return self.values

    @property
    def max_row_len(self) -> int:
        return int(self.mats[0].max_row_len)

    def status(self) -> list:
        return [fe_get_device_status(b, self.stream) for b in self.form_bufs] + \
               [fe_get_device_status(self.plan, self.stream)]


def fe_vector_plan(mesh: MeshView, n_phi: int, stream=None) -> torch.Tensor:
    """Dof -> (cell, i) adjacency of the dof map (symbolic phase of v^g = L b)."""
    lib = L.load()
    mv = mesh.struct()
    size = ctypes.c_size_t(0)
    check(lib.fe_vector_plan(ctypes.byref(mv), n_phi, None, ctypes.byref(size), _stream(stream)),
          "fe_vector_plan(size query)")
    plan = torch.empty(size.value, dtype=torch.uint8, device=mesh.coords.device)
    check(lib.fe_vector_plan(ctypes.byref(mv), n_phi, _ptr(plan), ctypes.byref(size),
                             _stream(stream)), "fe_vector_plan")
    return plan


def fe_action_vjp(desc: L.fe_form_desc, form_buf: torch.Tensor, mesh: MeshView,
                  vplan: torch.Tensor, mode: int, u: Optional[torch.Tensor],
                  v: Optional[torch.Tensor], y: Optional[torch.Tensor],
                  grad_u: Optional[torch.Tensor], grad_coeff: Optional[torch.Tensor],
                  workspace: Optional[torch.Tensor], stream=None,
                  ws_bytes: Optional[ctypes.c_size_t] = None) -> int:
    mv = mesh.struct()
    wb = ws_bytes if ws_bytes is not None else ctypes.c_size_t(
        0 if workspace is None else workspace.numel())
    return L.load().fe_action_vjp(ctypes.byref(desc), _ptr(form_buf), ctypes.byref(mv),
                                  _ptr(vplan), mode, _ptr(u), _ptr(v), _ptr(y), _ptr(grad_u),
                                  _ptr(grad_coeff), _ptr(workspace), ctypes.byref(wb),
                                  _stream(stream))


class Action:
    """y = A(z) u of one form on one mesh, and its vector-Jacobian product:
    prepares the form buffer and the vector plan once, sizes the workspace."""

    def __init__(self, mesh: MeshView, desc: L.fe_form_desc, stream=None):
        self.mesh, self.desc, self.stream = mesh, desc, stream
        dev = mesh.coords.device
        self.form_buf = fe_form_prepare(desc, dev, stream)
        self.n_phi = int(mesh.dofmap.shape[1])
        self.vplan = fe_vector_plan(mesh, self.n_phi, stream)
        self.dtype = torch.float64 if desc.precision == L.FE_FP64 else torch.float32
        sizes = []
        for mode, gz in ((L.FE_ACTION, False), (L.FE_VJP, True)):
            wb = ctypes.c_size_t(0)
            dummy = self.form_buf if gz else None
            check(fe_action_vjp(desc, self.form_buf, mesh, self.vplan, mode, None, None, None,
                                None, dummy, None, stream, wb), "fe_action_vjp(size query)")
            sizes.append(wb.value)
        self.workspace = torch.empty(max(sizes), dtype=torch.uint8, device=dev)

    def _vec(self, x: torch.Tensor) -> torch.Tensor:
        if x.dtype != self.dtype or not x.is_contiguous() or x.numel() != self.mesh.n_dofs:
            raise ValueError(f"expected a contiguous {self.dtype} vector of {self.mesh.n_dofs}")
        return x

    def apply(self, u: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y = A(z) u (FE_ACTION)."""
        u = self._vec(u)
        y = torch.empty_like(u) if out is None else out
        check(fe_action_vjp(self.desc, self.form_buf, self.mesh, self.vplan, L.FE_ACTION, u, None,
                            y, None, None, self.workspace, self.stream), "fe_action_vjp(ACTION)")
        return y

    def vjp(self, u: torch.Tensor, v: torch.Tensor, want_coeff: bool = True):
        """(grad_u, grad_coeff) for the cotangent v of y = A(z) u (FE_VJP);
        grad_coeff is None without a coefficient or when not wanted."""
        v = self._vec(v)
        gu = torch.empty_like(v)
        gz = None
        if want_coeff and self.desc.has_coeff:
            gz = torch.empty_like(v)
            u = self._vec(u)
        check(fe_action_vjp(self.desc, self.form_buf, self.mesh, self.vplan, L.FE_VJP,
                            u if gz is not None else None, v, None, gu, gz, self.workspace,
                            self.stream), "fe_action_vjp(VJP)")
        return gu, gz


class ActionFunction(torch.autograd.Function):
    """y = A(z) u with gradients for u and for the nodal coefficient z.

    The coefficient values live in ``action.mesh.coeff`` (the mesh view the
    library reads); the ``coeff`` argument must be that tensor, so that
    autograd can route its gradient.  Forward runs FE_ACTION, backward
    FE_VJP; both are the library's kernels."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, coeff: Optional[torch.Tensor], action: "Action"):
        if coeff is not None and coeff.data_ptr() != action.mesh.coeff.data_ptr():
            raise ValueError("coeff must be the coefficient tensor of the action's mesh")
        ctx.action = action
        ctx.save_for_backward(u)
        return action.apply(u.detach().contiguous())

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        (u,) = ctx.saved_tensors
        action = ctx.action
        want_z = ctx.needs_input_grad[1]
        gu, gz = action.vjp(u.detach().contiguous(), gy.detach().to(action.dtype).contiguous(),
                            want_coeff=want_z)
        if gz is not None:
            gz = gz.to(torch.float64)
        return (gu if ctx.needs_input_grad[0] else None), gz, None


def fe_cell_kernels_tile(desc: L.fe_form_desc, form_buf: torch.Tensor, mesh: MeshView,
                         A_local: torch.Tensor, tile: int, stream=None) -> None:
    mv = mesh.struct()
    check(L.load().fe_cell_kernels_tile(ctypes.byref(desc), _ptr(form_buf), ctypes.byref(mv),
                                        _ptr(A_local), int(tile), _stream(stream)),
          "fe_cell_kernels_tile")


def fe_tune_cell_kernels(desc: L.fe_form_desc, form_buf: torch.Tensor, mesh: MeshView,
                         A_local: torch.Tensor, reps: int = 3, stream=None):
    """(best tile, per-tile ms with -1 where a tile does not apply)."""
    mv = mesh.struct()
    best = ctypes.c_int32(-1)
    times = (ctypes.c_float * 10)()
    check(L.load().fe_tune_cell_kernels(ctypes.byref(desc), _ptr(form_buf), ctypes.byref(mv),
                                        _ptr(A_local), int(reps), ctypes.byref(best),
                                        ctypes.cast(times, ctypes.c_void_p), _stream(stream)),
          "fe_tune_cell_kernels")
    return int(best.value), [float(t) for t in times]


def fe_dg_pattern(n_cells: Sequence[int], n_phi: Sequence[int], device="cuda", stream=None):
    """(row_ptr int64 [n_dofs+1], col_idx int32 [nnz], nnz) of the block-diagonal
    CSR of a discontinuous space over degree blocks."""
    lib = L.load()
    nb = len(n_cells)
    nc = (ctypes.c_int64 * nb)(*[int(x) for x in n_cells])
    npi = (ctypes.c_int32 * nb)(*[int(x) for x in n_phi])
    nnz = ctypes.c_int64(0)
    check(lib.fe_dg_pattern(nb, ctypes.cast(nc, ctypes.c_void_p), ctypes.cast(npi, ctypes.c_void_p),
                            None, None, ctypes.byref(nnz), None), "fe_dg_pattern(size query)")
    n_dofs = sum(int(c) * int(p) for c, p in zip(n_cells, n_phi))
    row_ptr = torch.empty(n_dofs + 1, dtype=torch.int64, device=device)
    col_idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=device)
    check(lib.fe_dg_pattern(nb, ctypes.cast(nc, ctypes.c_void_p), ctypes.cast(npi, ctypes.c_void_p),
                            _ptr(row_ptr), _ptr(col_idx), ctypes.byref(nnz), _stream(stream)),
          "fe_dg_pattern")
    return row_ptr, col_idx, int(nnz.value)


class MixedDegree:
    """One form over the degree blocks of a mixed-degree discontinuous mesh,
    assembled into one block-diagonal CSR matrix.

    ``blocks``: (degree, quad_degree, cell_coords [n][4][3], dofmap [n][n_phi])
    per block, dofs numbered block-locally (the library places block b after
    blocks 0..b-1).  The numeric phase is one fe_cell_kernels_tile call per
    block, each writing its cells' local matrices into its slice of the CSR
    values; ``tune()`` picks every block's tile with fe_tune_cell_kernels and
    ``capture()`` records the calls of all blocks in one HIP graph, so that
    ``numeric()`` is a single graph launch.  In the graph the blocks can run
    on several streams (``groups``: lists of degrees, one stream each, a
    fork and a join): the small blocks' kernels then share the compute
    units with the large blocks' kernels, which leave registers and LDS free
    (one wave per SIMD at P7 and P8); the blocks write disjoint slices of
    the values."""

    def __init__(self, blocks, form: str = "mass", precision: str = "fp16", stream=None):
        self.stream = stream
        self.blocks = []
        n_cells, n_phi = [], []
        for (p, q, coords, dofmap) in blocks:
            mv = MeshView.from_numpy(coords, dofmap, max(int(np.asarray(dofmap).size), 1))
            desc = form_desc(3, p, q, form, precision)
            self.blocks.append({"degree": p, "mesh": mv, "desc": desc,
                                "form_buf": fe_form_prepare(desc, "cuda", stream), "tile": -1})
            n_cells.append(mv.n_cells)
            n_phi.append(int(np.asarray(dofmap).shape[1]))
        self.row_ptr, self.col_idx, self.nnz = fe_dg_pattern(n_cells, n_phi, "cuda", stream)
        dt = torch.float64 if precision == "fp64" else torch.float32
        self.values = torch.empty(max(self.nnz, 1), dtype=dt, device="cuda")
        off = 0
        for b, nc, npi in zip(self.blocks, n_cells, n_phi):
            b["values"] = self.values[off:off + nc * npi * npi]
            off += nc * npi * npi
        self.graph = None

    def tune(self, reps: int = 3) -> list:
        """Autotune every block's tile; returns (degree, tile, per-tile ms)."""
        out = []
        for b in self.blocks:
            if b["mesh"].n_cells == 0:
                continue
            b["tile"], times = fe_tune_cell_kernels(b["desc"], b["form_buf"], b["mesh"],
                                                    b["values"], reps, self.stream)
            out.append((b["degree"], b["tile"], times))
        self.graph = None
        return out

    def numeric_eager(self) -> torch.Tensor:
        self._launch(self.blocks)
        return self.values

    def _launch(self, blocks) -> None:
        for b in blocks:
            if b["mesh"].n_cells > 0:
                fe_cell_kernels_tile(b["desc"], b["form_buf"], b["mesh"], b["values"], b["tile"],
                                     self.stream)

    def capture(self, groups=((6, 7, 8), (1, 2, 3, 4, 5))) -> None:
        """Record the blocks' calls in one graph: the blocks of groups[0] on
        torch's current stream, each further group on a stream of its own
        that forks from it and joins it again, each group's blocks in the
        order of its degrees; degrees in no group run last on the current
        stream, and one group (or an own stream of the assembly, which the
        library must launch on) means one stream."""
        self.numeric_eager()                 # first launches outside the capture
        torch.cuda.synchronize()
        placed = {d for grp in groups for d in grp}
        parts = [[b for d in grp for b in self.blocks if b["degree"] == d] for grp in groups]
        parts[0] += [b for b in self.blocks if b["degree"] not in placed]
        parts = [p for p in parts if p]
        fork = self.stream is None and len(parts) > 1
        sides = [torch.cuda.Stream() for _ in parts[1:]] if fork else []
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            if fork:
                main = torch.cuda.current_stream()
                for s, p in zip(sides, parts[1:]):
                    s.wait_stream(main)
                    with torch.cuda.stream(s):
                        self._launch(p)
                self._launch(parts[0])
                for s in sides:
                    main.wait_stream(s)
            else:
                self.numeric_eager()
        self.graph = g
        self._sides = sides

    def numeric(self) -> torch.Tensor:
        if self.graph is None:
            return self.numeric_eager()
        self.graph.replay()
        return self.values

    def status(self) -> list:
        return [fe_get_device_status(b["form_buf"], self.stream) for b in self.blocks]
