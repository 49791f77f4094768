"""Seeded synthetic simplex meshes, dof maps and coefficient nodal values.

The paper measures on unstructured Gmsh meshes that are not available here
(Section 5.1); these generators stand in for them with meshes of the same
cell type (triangles and tetrahedra), polynomial degrees and cell counts well
above the paper's cache-spill cap.

Conventions (the reference simplex is the one of Section 5.1, vertices
0, e_1, ..., e_d):

* ``kuhn_mesh`` splits the unit square/cube into n^d boxes and every box into
  d! simplices, one per permutation s of the axes: v_0 = box corner,
  v_k = v_{k-1} + h e_{s_k}.  The split is conforming.  Boxes are numbered
  lexicographically (x fastest); inside a box, simplices follow
  ``itertools.permutations`` order.  Local vertex k corresponds to the
  reference vertex e_k (k >= 1) and vertex 0 to the origin.
* Local dofs of the degree-p Lagrange element sit on the principal lattice
  X_alpha = alpha / p, |alpha| <= p, ordered with alpha_d outermost and
  alpha_1 innermost (for p = 1 this is the vertex order above).
* Global continuous dofs are numbered by the node's position on the fine
  lattice of the unjittered mesh: i + (pn+1) j + (pn+1)^2 k.
* Only interior vertices are jittered, uniformly in [-r h, r h] per
  coordinate, from ``numpy.random.default_rng(seed)``.

Nothing here evaluates quadrature, basis functions, Jacobians or element
matrices.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Mesh:
    """A simplex mesh with per-cell vertex coordinates and a dof map."""

    d: int
    n: int                       # boxes per direction
    degree: int
    vertices: np.ndarray         # [n_v][d] float64 (jittered)
    cells: np.ndarray            # [n_K][d+1] int64 vertex ids
    lattice: np.ndarray          # [n_K][d+1][d] int64 unjittered vertex lattice coords (box units)
    cell_coords: np.ndarray      # [n_K][d+1][d] float64, per-cell copy (may be flattened)
    dofmap: np.ndarray           # [n_K][n_phi] int32
    n_dofs: int
    flattened: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    coeff: Optional[np.ndarray] = None   # [n_dofs] float64 nodal coefficient values

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_phi(self) -> int:
        return int(self.dofmap.shape[1])


def lattice_multi_indices(d: int, p: int) -> np.ndarray:
    """Multi-indices alpha (|alpha| <= p) in local dof order, shape [n_phi][d]."""
    out = []
    if d == 2:
        for a2 in range(p + 1):
            for a1 in range(p + 1 - a2):
                out.append((a1, a2))
    elif d == 3:
        for a3 in range(p + 1):
            for a2 in range(p + 1 - a3):
                for a1 in range(p + 1 - a3 - a2):
                    out.append((a1, a2, a3))
    else:
        raise ValueError("d must be 2 or 3")
    return np.asarray(out, dtype=np.int64).reshape(-1, d)


def _lex_points(m: int, d: int) -> np.ndarray:
    """All integer points of {0..m-1}^d, first coordinate fastest."""
    idx = np.arange(m ** d, dtype=np.int64)
    return np.stack([(idx // (m ** a)) % m for a in range(d)], axis=1)


def kuhn_mesh(d: int, n: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Unjittered Kuhn split of the unit box.

    Returns (vertices [n_v][d], cells [n_K][d+1], lattice [n_K][d+1][d]).
    """
    if d not in (2, 3):
        raise ValueError("d must be 2 or 3")
    nv = n + 1
    lat_v = _lex_points(nv, d)                 # vertex id = i + nv j (+ nv^2 k)
    vertices = lat_v.astype(np.float64) / n
    box = _lex_points(n, d)                    # box id, x fastest
    perms = list(itertools.permutations(range(d)))
    n_box = box.shape[0]
    lattice = np.zeros((n_box, len(perms), d + 1, d), dtype=np.int64)
    for pi, perm in enumerate(perms):
        cur = box.copy()
        lattice[:, pi, 0, :] = cur
        for k, ax in enumerate(perm):
            cur = cur.copy()
            cur[:, ax] += 1
            lattice[:, pi, k + 1, :] = cur
    lattice = lattice.reshape(n_box * len(perms), d + 1, d)
    strides = nv ** np.arange(d)
    cells = (lattice * strides).sum(axis=-1)
    return vertices, cells.astype(np.int64), lattice


def _orientation(x: np.ndarray) -> np.ndarray:
    """Sign of the simplex orientation (scalar triple / cross product), [n_K]."""
    e = x[:, 1:, :] - x[:, :1, :]
    if x.shape[2] == 2:
        o = e[:, 0, 0] * e[:, 1, 1] - e[:, 0, 1] * e[:, 1, 0]
    else:
        o = np.einsum("ij,ij->i", e[:, 0, :], np.cross(e[:, 1, :], e[:, 2, :]))
    return np.sign(o)


def jitter_interior(vertices: np.ndarray, n: int, r: float, seed: int,
                    cells: Optional[np.ndarray] = None) -> np.ndarray:
    """Move every interior vertex by i.i.d. U[-r h, r h] per coordinate.

    With ``cells`` given, vertices of any cell whose orientation flipped are
    redrawn from the same stream until no cell is inverted, so the jittered
    mesh stays a valid tessellation (at r = 0.25 in 3D a few cells in 10^5
    would otherwise invert).
    """
    if r == 0.0:
        return vertices.copy()
    h = 1.0 / n
    eps = 0.5 * h
    interior = np.all((vertices > eps) & (vertices < 1.0 - eps), axis=1)
    rng = np.random.default_rng(seed)
    out = vertices.copy()
    idx = np.nonzero(interior)[0]
    out[idx] += rng.uniform(-r * h, r * h, size=(idx.size, vertices.shape[1]))
    if cells is None:
        return out
    ref = _orientation(vertices[cells])
    for _ in range(100):
        bad = np.nonzero(_orientation(out[cells]) != ref)[0]
        if bad.size == 0:
            return out
        redo = np.unique(cells[bad].ravel())
        redo = redo[interior[redo]]
        out[redo] = vertices[redo] + rng.uniform(-r * h, r * h, size=(redo.size, vertices.shape[1]))
    raise RuntimeError("jitter could not avoid inverted cells")


def flatten_cells(cell_coords: np.ndarray, fraction: float, aspect: float, seed: int):
    """Flatten a seeded subset of cells in a per-cell copy of the coordinates.

    For each chosen cell the last vertex is moved along the unit normal of the
    opposite facet until its distance to that facet's hyperplane equals
    ``longest edge of the unflattened cell / aspect`` (same side as before).  Topology and dof map are
    unchanged, so geometry becomes non-conforming on purpose.
    Returns (new_coords, chosen cell ids).
    """
    nk, dp1, d = cell_coords.shape
    count = int(math.floor(fraction * nk))
    rng = np.random.default_rng(seed)
    chosen = np.sort(rng.choice(nk, size=count, replace=False))
    out = cell_coords.copy()
    x = out[chosen]
    base = x[:, 0, :]
    if d == 3:
        nrm = np.cross(x[:, 1, :] - base, x[:, 2, :] - base)
    else:
        e = x[:, 1, :] - base
        nrm = np.stack([-e[:, 1], e[:, 0]], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    longest = np.zeros(count)
    for a in range(dp1):
        for b in range(a + 1, dp1):
            longest = np.maximum(longest, np.linalg.norm(x[:, a, :] - x[:, b, :], axis=1))
    alt = np.einsum("ij,ij->i", x[:, -1, :] - base, nrm)
    target = np.sign(alt) * longest / aspect
    x[:, -1, :] -= (alt - target)[:, None] * nrm
    out[chosen] = x
    return out, chosen


def lattice_dofmap(lattice: np.ndarray, n: int, p: int) -> tuple[np.ndarray, int]:
    """Continuous degree-p Lagrange dof map on the fine lattice (pn+1)^d."""
    nk, dp1, d = lattice.shape
    alpha = lattice_multi_indices(d, p)                    # [n_phi][d]
    v0 = lattice[:, 0, :]                                   # [n_K][d]
    edges = lattice[:, 1:, :] - v0[:, None, :]              # [n_K][d][d]
    pos = p * v0[:, None, :] + np.einsum("ai,kij->kaj", alpha, edges)
    N = p * n + 1
    strides = N ** np.arange(d)
    dof = (pos * strides).sum(axis=-1)
    return dof.astype(np.int32), int(N ** d)


def dg_dofmap(n_cells: int, n_phi: int) -> tuple[np.ndarray, int]:
    """Broken (discontinuous) dof map: cell offset plus local index."""
    dof = np.arange(n_cells * n_phi, dtype=np.int64).reshape(n_cells, n_phi)
    return dof.astype(np.int32), int(n_cells * n_phi)


def nodal_values(cell_coords: np.ndarray, dofmap: np.ndarray, n_dofs: int, p: int,
                 fn: Callable[[np.ndarray], np.ndarray]) -> np.ndarray:
    """Values of ``fn`` at the physical Lagrange nodes, indexed by global dof.

    The node of local multi-index alpha sits at sum_i lambda_i x^i with
    lambda_i = alpha_i / p (i >= 1) and lambda_0 = 1 - sum.  On a conforming
    affine mesh every cell sharing a node places it at the same point (up to
    rounding), so any writer gives the same value.
    """
    nk, dp1, d = cell_coords.shape
    alpha = lattice_multi_indices(d, p).astype(np.float64) / p
    lam = np.concatenate([1.0 - alpha.sum(axis=1, keepdims=True), alpha], axis=1)
    pts = np.einsum("ai,kij->kaj", lam, cell_coords)        # [n_K][n_phi][d]
    vals = fn(pts.reshape(-1, d))
    out = np.zeros(n_dofs, dtype=np.float64)
    out[dofmap.reshape(-1).astype(np.int64)] = vals
    return out


def kappa_c3(x: np.ndarray) -> np.ndarray:
    """kappa(x, y, z) = exp(sin(2 pi x) cos(2 pi y) z)."""
    return np.exp(np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1]) * x[:, 2])


def normal_vector(n: int, seed: int) -> np.ndarray:
    """n samples of N(0, 1) from numpy's PCG64 stream ``seed``, rounded to FP32
    (the FE functions u, v of the action and adjoint workload)."""
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)


# Workload recipes.  Sizes follow the five benchmark configurations; ``scale``
# replaces the box count for reduced test sizes.
CONFIGS = {
    "c1": dict(d=2, n=32, degree=1, quad_degree=0, jitter=0.2, seed=0,
               flatten=0.0, forms=("stiffness",), coeff=None),
    "c2": dict(d=3, n=24, degree=4, quad_degree=8, jitter=0.25, seed=0,
               flatten=0.05, flatten_seed=1, forms=("mass", "stiffness"), coeff=None),
    "c3": dict(d=3, n=32, degree=6, quad_degree=14, jitter=0.25, seed=0,
               flatten=0.0, forms=("stiffness",), coeff="kappa"),
    # action y = A(kappa) u and its adjoint on the c3 mesh and coefficient,
    # u and v drawn by normal_vector with seeds 3 and 4
    "c5": dict(d=3, n=32, degree=6, quad_degree=14, jitter=0.25, seed=0,
               flatten=0.0, forms=("stiffness",), coeff="kappa", u_seed=3, v_seed=4),
}


def config_mesh(name: str, n: Optional[int] = None, degree: Optional[int] = None,
                flatten: Optional[float] = None) -> Mesh:
    """Build the mesh of a workload recipe (optionally with fewer boxes)."""
    cfg = CONFIGS[name]
    d = cfg["d"]
    n = cfg["n"] if n is None else n
    p = cfg["degree"] if degree is None else degree
    verts, cells, lattice = kuhn_mesh(d, n)
    verts = jitter_interior(verts, n, cfg["jitter"], cfg["seed"], cells)
    cell_coords = verts[cells]                       # [n_K][d+1][d]
    dofmap, n_dofs = lattice_dofmap(lattice, n, p)
    coeff = None
    if cfg["coeff"] == "kappa":
        coeff = nodal_values(cell_coords, dofmap, n_dofs, p, kappa_c3)
    frac = cfg["flatten"] if flatten is None else flatten
    flat = np.zeros(0, np.int64)
    if frac > 0.0:
        cell_coords, flat = flatten_cells(cell_coords, frac, 1e3, cfg["flatten_seed"])
    return Mesh(d=d, n=n, degree=p, vertices=verts, cells=cells, lattice=lattice,
                cell_coords=np.ascontiguousarray(cell_coords), dofmap=np.ascontiguousarray(dofmap),
                n_dofs=n_dofs, flattened=flat, coeff=coeff)


@dataclass
class DegreeBlock:
    """Cells of one degree of a mixed-degree mesh, with a discontinuous dof
    map numbered block-locally (dof of local index i in block cell K:
    K n_phi + i); the block's dofs follow those of the earlier blocks."""

    degree: int
    quad_degree: int
    cell_coords: np.ndarray      # [n_K][d+1][d] float64
    dofmap: np.ndarray           # [n_K][n_phi] int32, block-local numbering
    n_dofs: int
    dof_offset: int              # first global dof of the block
    nnz_offset: int              # first CSR entry of the block
    cell_ids: np.ndarray         # [n_K] indices of the cells in the source mesh

    @property
    def n_cells(self) -> int:
        return int(self.cell_coords.shape[0])

    @property
    def n_phi(self) -> int:
        return int(self.dofmap.shape[1])


def mixed_degree_blocks(n: int = 41, n_cells: int = 400_000, degrees=range(1, 9),
                        jitter: float = 0.25, seed: int = 0, degree_seed: int = 2,
                        cell_limit: Optional[int] = None) -> list:
    """The mixed-degree workload: the first ``n_cells`` tetrahedra of the
    jittered n^3 x 6 Kuhn mesh, a degree p drawn per cell with P(p) ~ 1/p
    (``numpy.random.default_rng(degree_seed)``), quadrature degree 2p, and
    the cells grouped into one contiguous block per degree (degree order,
    source order inside a block) with a discontinuous dof map, so the global
    matrix is block diagonal with sum_K n_phi(p_K)^2 entries.
    ``cell_limit`` keeps only the first cells (reduced test sizes)."""
    verts, cells, _ = kuhn_mesh(3, n)
    verts = jitter_interior(verts, n, jitter, seed, cells)
    cc = verts[cells[:n_cells]]
    degs = np.asarray(list(degrees))
    prob = 1.0 / degs
    prob /= prob.sum()
    p_cell = np.random.default_rng(degree_seed).choice(degs, size=cc.shape[0], p=prob)
    if cell_limit is not None:
        cc, p_cell = cc[:cell_limit], p_cell[:cell_limit]
    blocks, dof_off, nnz_off = [], 0, 0
    for p in degs:
        ids = np.flatnonzero(p_cell == p)
        n_phi = math.comb(p + 3, 3)
        dm, nd = dg_dofmap(ids.size, n_phi)
        blocks.append(DegreeBlock(degree=int(p), quad_degree=int(2 * p),
                                  cell_coords=np.ascontiguousarray(cc[ids]), dofmap=dm,
                                  n_dofs=nd, dof_offset=dof_off, nnz_offset=nnz_off,
                                  cell_ids=ids))
        dof_off += nd
        nnz_off += ids.size * n_phi * n_phi
    return blocks


def hex_mesh(n: int, degree: int, jitter: float = 0.25, seed: int = 0) -> Mesh:
    """n^3 hexahedra of the unit cube (box x fastest), interior vertices
    jittered by U[-r h, r h] per coordinate (trilinear cells); the cell's
    vertex v is its box corner (v & 1, (v >> 1) & 1, (v >> 2) & 1).  Dof map
    of Q_p on the fine lattice (pn+1)^3: local (i, j, k) -> global
    (p bx + i) + N (p by + j) + N^2 (p bz + k), local index i + (p+1)(j + (p+1)k)."""
    nv = n + 1
    lat_v = _lex_points(nv, 3)
    verts = lat_v.astype(np.float64) / n
    if jitter > 0.0:
        verts = jitter_interior(verts, n, jitter, seed)
    box = _lex_points(n, 3)
    corners = np.array([[(v >> e) & 1 for e in range(3)] for v in range(8)])
    lattice = box[:, None, :] + corners[None, :, :]                      # [n^3][8][3]
    cells = (lattice * (nv ** np.arange(3))).sum(axis=-1)
    cell_coords = np.ascontiguousarray(verts[cells])
    p, N = degree, degree * n + 1
    loc = _lex_points(p + 1, 3)                                          # i fastest
    pos = p * box[:, None, :] + loc[None, :, :]
    dofmap = (pos * (N ** np.arange(3))).sum(axis=-1).astype(np.int32)
    return Mesh(d=3, n=n, degree=p, vertices=verts, cells=cells, lattice=lattice,
                cell_coords=cell_coords, dofmap=np.ascontiguousarray(dofmap), n_dofs=int(N ** 3))
