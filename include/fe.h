/*
 * fe.h -- C ABI of the MI355X (gfx950) finite element cell-kernel and
 * assembly library.
 *
 * The library computes, for every cell K of a mesh of affine simplices
 * (triangles, tetrahedra) or trilinear hexahedra, the local element matrix
 * of the mass or Poisson (stiffness) form with an optional coefficient z in
 * the same Lagrange space,
 *
 *     A_K = sum_{s,t} B_s C_st B_t^T,   C_st = diag_q(w_q z(X_q) G_st)
 *
 * (Croci & Wells, Section 3.1, eq. triple_products; Algorithm 1 in
 * Section 3.2), and assembles the global matrix A^g = L D L^T into CSR
 * (Section 3.3).  B holds reference basis values (mass) or gradients
 * (Poisson) at the quadrature points; G = |det J| (mass) or
 * G = |det J| J^{-1} J^{-T} (Poisson) is the geometry tensor (Section 4.2).
 *
 * Conventions shared by every call:
 *   - Every function returns an fe_status (0 = success).  Argument errors are
 *     detected on the host before anything is enqueued; outputs are then
 *     left untouched.  No C++ exception crosses this boundary.
 *   - The caller owns all memory.  Device buffers are allocated by the
 *     caller (for instance through PyTorch) and passed as plain pointers;
 *     sizes of library-internal buffers are obtained by a size query
 *     (NULL buffer, non-NULL size pointer).  The library never allocates or
 *     frees device memory.
 *   - Device work is enqueued on the caller's stream (hipStream_t passed as
 *     void*; NULL = default stream).  Calls do not synchronise unless stated.
 *   - Calls hold no global state and may be issued from several host threads
 *     on distinct buffers.
 *   - Floating-point results of the reduced/mixed precision modes are
 *     deterministic for a given GPU, input and build: the numeric assembly
 *     sums every CSR entry in a fixed order.
 *
 * Simplex geometry is affine: J, det J and G are constant on a cell,
 * computed once per cell (in FP64 by default: the geometry precision u_g of
 * List 1 is double).  Hexahedra are mapped trilinearly, so J, det J and G
 * vary over the cell and are evaluated in FP64 at every quadrature point.
 */
#ifndef FE_MI355X_FE_H
#define FE_MI355X_FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fe_status;

enum {
  FE_OK = 0,
  FE_EINVAL = -1,       /* bad argument: NULL pointer, size, range, dof index */
  FE_EUNSUPPORTED = -2, /* valid but not implemented: cell, degree, precision */
  FE_EOVERFLOW = -3,    /* an index would not fit its integer type */
  FE_EHIP = -4,         /* a HIP runtime call failed */
  FE_EDEGENERATE = -5,  /* a cell has det J == 0 or non-finite geometry */
  FE_ESIZE = -6         /* a caller buffer is smaller than the queried size */
};

/* Reference cells (Section 5.1): the triangle / tetrahedron with vertices
 * 0, e_1, ..., e_d (the value equals the dimension d), and the hexahedron
 * (boxed cell, value 8: its vertex count) on the unit cube [0,1]^3, mapped
 * trilinearly; its cell_coords are [n_cells][8][3], vertex v at the reference
 * corner (v & 1, (v >> 1) & 1, (v >> 2) & 1).  Hexahedra: Lagrange Q_p on the
 * equispaced lattice (n_phi = (p+1)^3, local index i + (p+1)(j + (p+1)k)),
 * p <= 7, tensor Gauss-Legendre quadrature; J, |det J| and the Poisson
 * tensor G vary over the cell and enter per quadrature point (FP64).  The
 * Poisson form keeps G of a batch of 16 cells at every point in LDS in the
 * arithmetic type of H: it is available up to Q7 in FE_FP16_ACC32, Q6 in the
 * single-precision modes and Q4 in FE_FP64 (FE_EUNSUPPORTED beyond). */
enum { FE_TRIANGLE = 2, FE_TETRAHEDRON = 3, FE_HEXAHEDRON = 8 };

/* Forms of Section 3.1. */
enum { FE_MASS = 0, FE_STIFFNESS = 1 };

/* Arithmetic of the contraction A = B^T H (List 1, Section 4.5):
 *   FE_FP64            everything in double (u_s = u_q = u_g = FP64)
 *   FE_FP32            B and H in single, single accumulation
 *   FE_FP16_ACC32      B, the weighted table w_q B and the geometry factors
 *                      stored in half and H computed in half (u_s = FP16, as
 *                      in List 1), products and accumulation in single on
 *                      the matrix cores (u_q)
 *   FE_BF16_ACC32      B and H stored in bfloat16; H formed in single and
 *                      rounded once
 *   FE_SPLITFP16_ACC32 B and H each stored as a pair hi + 2^-11 lo of halves
 *                      (H formed in single first); three products
 *                      hi*hi + 2^-11 (hi*lo + lo*hi), single accumulation.
 * In all modes geometry is FP64 (u_g). */
enum {
  FE_FP64 = 0,
  FE_FP32 = 1,
  FE_FP16_ACC32 = 2,
  FE_BF16_ACC32 = 3,
  FE_SPLITFP16_ACC32 = 4
};

/* Geometry precision u_g (Section 4.2; the per-cell choice remark of
 * Section 5.2):
 *   FE_GEOM_FP64  J, det J, J^{-1} and G in double (the default)
 *   FE_GEOM_FP32  in single, from the coordinates rounded to single
 *   FE_GEOM_AUTO  in single, recomputed in double for cells whose single
 *                 result is degenerate or whose condition estimate
 *                 ||J||_F ||adj J||_F / |det J| exceeds 2^10 (the single
 *                 error kappa u_32 then stays below an eighth of the FP16
 *                 unit roundoff).
 * All forms of one fe_assemble_csr call must use the same mode. */
enum { FE_GEOM_FP64 = 0, FE_GEOM_FP32 = 1, FE_GEOM_AUTO = 2 };

/* Phases of fe_assemble_csr. */
enum {
  FE_SYMBOLIC_COUNT = 0,
  FE_SYMBOLIC_FILL = 1,
  FE_NUMERIC = 2,
  FE_NUMERIC_GATHER = 3,
  FE_NUMERIC_GEOMETRY = 4, /* first half of the fused FE_NUMERIC */
  FE_NUMERIC_FUSED = 5,    /* second half of the fused FE_NUMERIC */
  FE_NUMERIC_LOCAL = 6,    /* first half of FE_NUMERIC_GATHER: local matrices */
  FE_NUMERIC_ASSEMBLE = 7  /* second half of FE_NUMERIC_GATHER: the row gather */
};

typedef struct fe_form_desc {
  int32_t cell;           /* FE_TRIANGLE, FE_TETRAHEDRON or FE_HEXAHEDRON      */
  int32_t degree;         /* Lagrange degree p, 1 <= p <= 8                     */
  int32_t quad_degree;    /* q >= 0: floor(q/2)+1 collapsed Gauss-Jacobi points
                             per direction, at most 9 (q <= 17)                 */
  int32_t form;           /* FE_MASS or FE_STIFFNESS                            */
  int32_t has_coeff;      /* 1: multiply by z(X_q) = sum_k z_k phi_k(X_q)      */
  int32_t precision;      /* FE_FP64 ... FE_SPLITFP16_ACC32                     */
  int32_t geom_precision; /* FE_GEOM_FP64, FE_GEOM_FP32 or FE_GEOM_AUTO          */
} fe_form_desc;

typedef struct fe_mesh_view {
  int64_t n_cells;
  const double *cell_coords; /* device [n_cells][d+1][d] FP64; vertex k <-> e_k */
  const int32_t *dofmap;     /* device [n_cells][n_phi], entries in [0, n_dofs) */
  int64_t n_dofs;
  const double *coeff;       /* device [n_dofs] nodal values z, or NULL         */
} fe_mesh_view;

typedef struct fe_csr {
  int64_t n_rows;   /* = n_dofs                                               */
  int64_t nnz;      /* written by FE_SYMBOLIC_COUNT                            */
  int64_t max_row_len; /* written by FE_SYMBOLIC_COUNT: longest row           */
  int64_t schedule; /* written by FE_SYMBOLIC_FILL: owner tasks of the fused
                       numeric schedule, 0 when none was built              */
  int32_t schedule_span; /* written by FE_SYMBOLIC_FILL: CSR entries per task
                            of that schedule (1024, or 2048 when every form
                            of the FILL call was an FP16 hexahedral form)    */
  int32_t schedule_elt;  /* written by FE_SYMBOLIC_FILL: bytes per value of
                            the forms of the FILL call (8 FP64, else 4); the
                            schedule's record layout depends on it           */
  int64_t *row_ptr; /* device [n_rows+1]                                       */
  int32_t *col_idx; /* device [nnz], ascending and unique per row              */
  void *values;     /* device [nnz], double for FE_FP64 else float             */
} fe_csr;

/* ------------------------------------------------------------------------
 * fe_tabulate -- reference quadrature and basis tabulation (host, FP64).
 *
 * Algorithm 1 step 1; the tables B of Section 3.1 (B_skq = d_s phi_k(X_q) or
 * phi_k(X_q)).  Quadrature: m = floor(q/2)+1 Gauss-Jacobi points per
 * direction on [0,1] with weights (1-t)^0, (1-t)^1, (1-t)^2, collapsed onto
 * the simplex (X = a(1-b)(1-c), Y = b(1-c), Z = c), a fastest.  Basis:
 * equispaced-lattice Lagrange functions in product form (Appendix A),
 * local order alpha_d outermost, alpha_1 innermost.
 *   n_phi, n_q : out, always written on success
 *   points     : out [n_q][d] or NULL
 *   weights    : out [n_q] or NULL
 *   table      : out [1 + d*nderiv][n_q][n_phi] or NULL: slab 0 = values,
 *                slab 1+s = d/dX_s (nderiv = 1)
 * Call with NULL buffers to query sizes.  Errors: FE_EINVAL (bad cell, p<1,
 * q<0, nderiv not 0/1, NULL size pointers), FE_EUNSUPPORTED (p > 8,
 * q > 17).  Synchronous; touches no device.
 * ------------------------------------------------------------------------ */
fe_status fe_tabulate(int32_t cell, int32_t degree, int32_t quad_degree, int32_t nderiv,
                      int32_t *n_phi, int32_t *n_q, double *points, double *weights,
                      double *table);

/* ------------------------------------------------------------------------
 * fe_form_prepare -- device copy of the tabulation in operand layout.
 *
 * Algorithm 1 step 1, device side: B rounded once from FP64 to the operand
 * format of f->precision (hi/lo pair for the split mode) and packed in the
 * lane order of the matrix-core instructions, the weighted table w_q B used
 * to form H = C B^T in single (double for FE_FP64), and, with a
 * coefficient, the value table used to evaluate z at the quadrature points.
 * FP32 and FP64 forms with n_phi <= 84 also carry the tables of the action
 * kernels (values and gradients in the lane order of fe_action_vjp, per
 * tile of 16 quadrature points, with the weights).
 * The buffer also holds a device status word (see fe_get_device_status).
 *   form_buf   : device buffer of *form_bytes bytes, or NULL for a size query
 *   form_bytes : in/out; on a query receives the required size; on a real
 *                call must be >= that size (else FE_ESIZE)
 * Synchronous with respect to the host (the upload is complete on return).
 * Errors: FE_EINVAL, FE_EUNSUPPORTED, FE_ESIZE, FE_EHIP.
 * ------------------------------------------------------------------------ */
fe_status fe_form_prepare(const fe_form_desc *f, void *form_buf, size_t *form_bytes,
                          void *stream);

/* ------------------------------------------------------------------------
 * fe_cell_kernels -- local element matrices of every cell (unassembled).
 *
 * Algorithm 1 steps 2-4 for all cells: FP64 geometry (J, det J, J^{-1},
 * G; Section 4.2), the coefficient at the quadrature points when
 * f->has_coeff (Lemma on FE function evaluation), H = C B^T formed on chip
 * and the contraction A = B^T H on the matrix cores, cells batched 16 at a
 * time along the N dimension (the cell batching of Section 3.1).
 *   form_buf : prepared by fe_form_prepare for the same *f
 *   A_local  : device [n_cells][n_phi][n_phi], row-major, row = first basis
 *              index; double for FE_FP64, float otherwise
 * Asynchronous.  A degenerate cell (det J == 0 or non-finite geometry)
 * yields NaN entries for that cell and sets FE_EDEGENERATE in the status
 * word of form_buf.  Errors: FE_EINVAL (NULL pointers, n_cells < 0, coeff
 * missing while f->has_coeff), FE_EUNSUPPORTED, FE_EHIP.
 * ------------------------------------------------------------------------ */
fe_status fe_cell_kernels(const fe_form_desc *f, const void *form_buf, const fe_mesh_view *m,
                          void *A_local, void *stream);

/* ------------------------------------------------------------------------
 * fe_cell_kernels_tile -- fe_cell_kernels with an explicit tile variant.
 *
 * tile = variant + 4 * occ, 0 <= tile < 8, tile 8, tile 9, or -1 for the
 * default:
 *   variant 0: 8-wave workgroups, B^T fragments and the weighted table
 *              staged in LDS (forms with at most 4 row tiles of 16 whose
 *              tables fit)
 *   variant 1: 4-wave workgroups, fragments staged in LDS
 *   variant 2: 4-wave workgroups, fragments and table read through the caches
 *   variant 3: 8-wave workgroups, fragments and table streamed through a
 *              double-buffered LDS ring one quadrature chunk at a time
 *              (not for FE_SPLITFP16_ACC32)
 *   occ 1    : twice the workgroups per compute unit of occ 0.
 *   tile 8   : the whole-cell kernel (one wave per cell, every quadrature
 *              chunk's B^T fragments shared through an LDS ring by the
 *              workgroup, only the tiles of one triangle of the symmetric
 *              matrix contracted) for FE_FP16_ACC32 tetrahedral forms
 *              without a coefficient: mass P5..P8, Poisson P6.
 *   tile 9   : the smallest FE_FP16_ACC32 mass forms without a coefficient
 *              (n_phi 3, 4, 6 or 10: P1, P2 tetrahedra, P1..P3 triangles,
 *              at most 128 quadrature points) on the vector ALUs, one
 *              thread per row of a local matrix (Section 3, Algorithm 1).
 * Tiles 0..7 sum every entry in the same order: results are bitwise
 * identical across them.  Tile 8 forms H from the fragments and per-point
 * products c_st(q) = w_q G_st rounded to half (the same precision, its own
 * rounding order): within the same error bound, not bitwise equal.  Tile 9
 * forms the same half H as tiles 0..7 and sums the exact products in
 * single in its own order: within the same bound, not bitwise equal.
 * FE_EUNSUPPORTED when the variant does not apply to the form; FE_EINVAL
 * for a tile out of range; otherwise as fe_cell_kernels.
 * ------------------------------------------------------------------------ */
fe_status fe_cell_kernels_tile(const fe_form_desc *f, const void *form_buf, const fe_mesh_view *m,
                               void *A_local, int32_t tile, void *stream);

/* ------------------------------------------------------------------------
 * fe_tune_cell_kernels -- autotuner of the cell-kernel tile for one form and
 * mesh: runs every tile variant that applies (one warm-up launch, then
 * `reps` timed launches with HIP events on the stream) and returns the
 * fastest in *best_tile; times_ms (NULL or [10]) receives the average time
 * per launch of each tile, -1 where the tile does not apply.  A_local is
 * overwritten (the result of the last tile run).  SYNCHRONISES the stream.
 * Errors: FE_EINVAL (reps < 1, NULL best_tile), FE_EUNSUPPORTED (no tile
 * applies), and those of fe_cell_kernels.
 * ------------------------------------------------------------------------ */
fe_status fe_tune_cell_kernels(const fe_form_desc *f, const void *form_buf, const fe_mesh_view *m,
                               void *A_local, int32_t reps, int32_t *best_tile, float *times_ms,
                               void *stream);

/* ------------------------------------------------------------------------
 * fe_dg_pattern -- CSR pattern of a discontinuous Lagrange space over
 * degree blocks (the mixed-degree mesh of Section 5 with its cells grouped
 * by degree): block b holds n_cells[b] cells of n_phi[b] dofs numbered
 * cell-major after the dofs of blocks 0..b-1, so the global matrix
 * A^g = L D L^T (Section 3.3) is block diagonal and the row-major local
 * matrices of the cells of block b, in cell order, are exactly its CSR
 * values from entry sum_{b' < b} n_cells[b'] n_phi[b']^2 on: the numeric
 * phase is fe_cell_kernels(_tile) per block writing into one values array.
 *   n_cells, n_phi : host [n_blocks]; 1 <= n_phi[b] <= 1024
 *   row_ptr  : device [n_dofs + 1] int64 (n_dofs = sum n_cells[b] n_phi[b])
 *   col_idx  : device [nnz] int32, ascending per row
 *   nnz      : out (host), sum n_cells[b] n_phi[b]^2; with row_ptr or col_idx
 *              NULL only nnz is computed (size query)
 * Asynchronous.  Errors: FE_EINVAL, FE_EOVERFLOW (n_dofs >= 2^31 - 1),
 * FE_EHIP.
 * ------------------------------------------------------------------------ */
fe_status fe_dg_pattern(int32_t n_blocks, const int64_t *n_cells, const int32_t *n_phi,
                        int64_t *row_ptr, int32_t *col_idx, int64_t *nnz, void *stream);

/* ------------------------------------------------------------------------
 * fe_assemble_csr -- global assembly A^g = L D L^T into CSR (Section 3.3).
 *
 * The CSR pattern is the set of pairs (dof(K,i), dof(K,j)) over all cells,
 * rows in dof order, columns ascending and unique, explicit zeros kept.  It
 * depends only on the dof map, so n_forms forms (for instance mass and
 * stiffness) sharing one mesh share one pattern and one plan.
 *
 *   forms[n_forms], form_bufs[n_forms] : 1 <= n_forms <= 4; every form must
 *       have the same cell and degree and all forms the same value type
 *       (all FE_FP64 or none)
 *   mats[n_forms] : output matrices; row_ptr/col_idx may be shared
 *   plan / plan_bytes : device scratch owned by the caller, sized by a query
 *       with plan == NULL; holds the dof-to-cell adjacency, the position of
 *       every local entry inside its CSR row and the fused schedule.  Its
 *       size depends on the mesh (n_cells, n_phi, n_dofs) and on the value
 *       type of the forms (FP64 or not: the schedule's record layout).  The
 *       schedule built by FE_SYMBOLIC_FILL serves only forms of the value
 *       type and task span of that call (mats[0].schedule_elt and
 *       schedule_span); FE_NUMERIC takes the gather for other forms.
 *   workspace / ws_bytes : device scratch for the numeric phase (local
 *       matrices of all forms for the gather, per-cell factors of H for the
 *       fused path), sized by a query with workspace == NULL.
 *
 * Phases:
 *   FE_SYMBOLIC_COUNT : fills mats[0].row_ptr and writes nnz and max_row_len
 *       into every mats[f].  SYNCHRONISES the stream (nnz is read back).
 *       FE_EOVERFLOW when a row holds 65536 or more entries.
 *   FE_SYMBOLIC_FILL  : fills mats[0].col_idx (sorted) and the plan: the
 *       position of every local entry inside its CSR row and, when every
 *       row fits one owner task (at most 1024 entries, 2048 when every form
 *       is an FP16 hexahedral form, and 64 incident (cell, local index)
 *       pairs), the row-ownership schedule of the fused
 *       numeric path; writes its task count into every mats[f].schedule.
 *       SYNCHRONISES the stream.
 *   FE_NUMERIC : writes the values of every form.  With a schedule
 *       (mats[0].schedule > 0, the mats of the FILL phase) and forms without
 *       a coefficient whose tables fit the on-chip memory, it runs per form a
 *       per-cell FP64 geometry pass and one fused kernel: every wave owns a
 *       range of CSR rows in LDS, computes the local rows A_K(j, :) of
 *       exactly the dofs it owns on the matrix cores and writes its rows
 *       once (hexahedral forms: the geometry pass also evaluates |det J| at
 *       every quadrature point).  Otherwise it runs the cell kernels into
 *       the workspace followed by the row gather.  Either way every entry's
 *       contributions are summed in the fixed order cell ascending and every
 *       value is written exactly once (no separate zero-fill).
 *       Asynchronous, never synchronises, bitwise repeatable.
 *   FE_NUMERIC_GATHER : as FE_NUMERIC but always through the workspace and
 *       the row gather (for comparison and testing).
 *   FE_NUMERIC_GEOMETRY, FE_NUMERIC_FUSED : the two halves of the fused
 *       FE_NUMERIC, for callers that keep the coordinates fixed over several
 *       assemblies or time the halves: GEOMETRY writes the per-cell factor
 *       records (for hexahedra also |det J| at every quadrature point) into
 *       the workspace, FUSED runs the fused kernels on the records the last
 *       GEOMETRY (or FE_NUMERIC) call left in that workspace.
 *       FE_EUNSUPPORTED when the fused path does not apply to every form;
 *       FE_EINVAL when the schedule was built for forms of another value
 *       type or task span (checked on the host before any launch).
 *   FE_NUMERIC_LOCAL, FE_NUMERIC_ASSEMBLE : the two halves of
 *       FE_NUMERIC_GATHER: LOCAL writes the local matrices of every form
 *       into the workspace, ASSEMBLE runs the row gather on what the last
 *       LOCAL (or FE_NUMERIC / FE_NUMERIC_GATHER) call left there.
 *   FP16 Poisson forms with a coefficient on P6 tetrahedra compute their
 *   local matrices with a whole-cell kernel (one wave per cell, symmetric
 *   tiles, the coefficient at the points evaluated first into the
 *   workspace); fe_cell_kernels keeps the batched cell kernel.
 * Errors: FE_EINVAL (NULL pointers, dof entries out of range are reported
 * through the status word of the plan), FE_ESIZE, FE_EUNSUPPORTED, FE_EHIP.
 * ------------------------------------------------------------------------ */
fe_status fe_assemble_csr(const fe_form_desc *forms, const void *const *form_bufs,
                          int32_t n_forms, const fe_mesh_view *m, int32_t phase,
                          fe_csr *mats, void *plan, size_t *plan_bytes, void *workspace,
                          size_t *ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * fe_assemble_csr_noalloc -- FE_NUMERIC of fe_assemble_csr without a
 * caller workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).
 *
 * Same arguments and results as fe_assemble_csr with phase FE_NUMERIC, for
 * forms that all take the fused row-ownership path (a schedule built by
 * FE_SYMBOLIC_FILL for these forms, no coefficient, tables that fit on
 * chip): the per-cell factor records of the fused path (and the per-point
 * factors of hexahedral mass forms) are kept in a scratch array inside the
 * library, 16 MiB per GPU (every GPU the library runs on holds its copy
 * until the process ends), instead of the caller's workspace.  The call
 * allocates nothing.  Calls that overlap on one GPU share that array and
 * race: serialise them (one stream, or events).  The array keeps the last
 * call's contents; every record is written before it is read.
 * Errors (on the host, before anything is enqueued): FE_ESIZE when the
 * records of these forms and cells exceed the 16 MiB (about 250,000 cells
 * for two forms); FE_EUNSUPPORTED when a form does not take the fused
 * path; otherwise those of fe_assemble_csr.
 * ------------------------------------------------------------------------ */
fe_status fe_assemble_csr_noalloc(const fe_form_desc *forms, const void *const *form_bufs,
                                  int32_t n_forms, const fe_mesh_view *m, fe_csr *mats,
                                  void *plan, void *stream);

/* Modes of fe_action_vjp. */
enum { FE_ACTION = 0, FE_VJP = 1 };

/* ------------------------------------------------------------------------
 * fe_vector_plan -- symbolic phase of vector assembly v^g = L b (Section
 * 3.3): the dof -> (cell, local index) adjacency of the dof map, every list
 * in cell-ascending order, so that the numeric sums of fe_action_vjp run in
 * a fixed order.
 *   n_phi : dofs per cell (the dof map's row length), 1 <= n_phi <= 256
 *   plan / plan_bytes : device buffer owned by the caller, sized by a query
 *       with plan == NULL; its size depends on n_cells, n_phi and n_dofs.
 * SYNCHRONISES the stream.  Errors: FE_EINVAL (NULL pointers, a dof entry
 * out of range), FE_EOVERFLOW (n_dofs >= 2^31 - 1), FE_ESIZE, FE_EHIP.
 * ------------------------------------------------------------------------ */
fe_status fe_vector_plan(const fe_mesh_view *m, int32_t n_phi, void *plan, size_t *plan_bytes,
                         void *stream);

/* ------------------------------------------------------------------------
 * fe_action_vjp -- the action y = A(z) u of the mass or Poisson form and its
 * vector-Jacobian product, matrix free (Algorithm 2, Section 3.2; the local
 * vectors v = sum_s B_s r_s with r_s = vstack_q(w_q z(X_q) (G grad u)_s),
 * assembled as v^g = L b, Section 3.3).
 *   mode FE_ACTION : y = A(z) u.  Reads u; writes y [n_dofs].
 *   mode FE_VJP    : for the cotangent v of y, grad_u = A(z)^T v (= A(z) v,
 *       both forms being symmetric) and, when grad_coeff != NULL (requires
 *       f->has_coeff), grad_coeff[m] = v^T (dA/dz_m) u
 *         = sum_K sum_{k: L(K,k) = m} sum_q phi_k(X_q) w_q g_K(q),
 *       g_K = (grad v_h)^T G (grad u_h) (Poisson) or |det J| v_h u_h (mass).
 *       Reads v (and u for grad_coeff).
 *   form_buf : prepared by fe_form_prepare for the same *f; precision
 *       FE_FP32 or FE_FP64 with n_phi <= 84 (else FE_EUNSUPPORTED)
 *   vplan    : from fe_vector_plan for the same mesh
 *   u, v, y, grad_u, grad_coeff : device [n_dofs], double for FE_FP64 else
 *       float.  Outputs are overwritten (every entry written once); each
 *       sums its contributions in the fixed order cell ascending.
 *   workspace / ws_bytes : local vectors, sized by a query with
 *       workspace == NULL (the size depends on the mode and on whether
 *       grad_coeff is requested).
 * Geometry is FP64 per cell, rounded once to the arithmetic type; the
 * coefficient is evaluated in that type.  Asynchronous, never synchronises.
 * A degenerate cell gives NaN contributions and sets FE_EDEGENERATE in the
 * status word of form_buf; a dof out of range or a plan of another mesh
 * sets FE_EINVAL there (fe_get_device_status).  Errors: FE_EINVAL,
 * FE_EUNSUPPORTED, FE_ESIZE, FE_EOVERFLOW, FE_EHIP.
 * ------------------------------------------------------------------------ */
fe_status fe_action_vjp(const fe_form_desc *f, const void *form_buf, const fe_mesh_view *m,
                        const void *vplan, int32_t mode, const void *u, const void *v, void *y,
                        void *grad_u, void *grad_coeff, void *workspace, size_t *ws_bytes,
                        void *stream);

/* ------------------------------------------------------------------------
 * fe_get_device_status -- read and clear the status word of a form buffer
 * or plan after the work that could set it.  Synchronises the stream.
 * Returns FE_OK, FE_EDEGENERATE (a degenerate cell was met) or FE_EINVAL
 * (a dof index was out of range), or FE_EHIP on a runtime failure.
 * ------------------------------------------------------------------------ */
fe_status fe_get_device_status(const void *form_buf_or_plan, void *stream);

/* Static English description of a status code. */
const char *fe_status_string(fe_status s);

/* Library version, for diagnostics: "fe-mi355x <major>.<minor>". */
const char *fe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_MI355X_FE_H */
