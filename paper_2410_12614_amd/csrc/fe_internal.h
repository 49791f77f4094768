// Internal declarations of the gfx950 finite element library (not part of the ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "fe.h"

#define FE_MAX_DEGREE 8
#define FE_MAX_QUAD_DEGREE 17
#define FE_MAX_BOX_DEGREE 7

namespace fe {

// ---- host tabulation (fe_tabulate.cpp) ----
void gauss_jacobi_01(int m, int alpha, double *t, double *w);
int simplex_dim(int d, int p);
void lattice_indices(int d, int p, std::vector<int> &out);
void lagrange_eval(int d, int p, const double *X, double *val, double *grad);

// Adjacency entries (dof -> incident (cell, local index) pairs) encode
// cell * 2^ADJ_BITS + i: local indices up to 1023 (Q_7 hexahedra: 512).
constexpr int ADJ_BITS = 10;
constexpr int64_t ADJ_MASK = (1 << ADJ_BITS) - 1;

// Device status word bits (stored in the first word of a form buffer or plan).
enum : int32_t { STATUS_DEGENERATE = 1, STATUS_BAD_DOF = 2 };

// Layout of a prepared form buffer.  Everything is derived from the form
// descriptor alone, so host launchers can recompute it without reading the
// device buffer.
//
// Operand conventions (K index k = s * n_q_pad + q, s < nd):
//   afrag   : B^T packed per 16x16xKSTEP matrix-core fragment,
//             [mt][ks][lane][KPL] with element B_s(q, i), i = 16 mt + lane % 16,
//             k = ks*KSTEP + (lane / 16) * KPL + e  (zero padding)
//   afrag_lo: split mode only, fl16((B - fl16(B)) * 2^11) in the same layout
//   wtab    : weighted table w_q B_t(q, j), [t][j][n_q_pad], t < NDT
//   vtab    : basis values phi_k(X_q), [n_q][n_phi] (coefficient evaluation)
//   wq      : quadrature weights w_q, [n_q_pad] double (zero padding)
//   act     : tables of the action kernels (FP32 and FP64 forms with
//             n_phi <= 84), one chunk of act_chunk elements per tile of 16
//             quadrature points qt, see fe_action.h (K-steps padded to
//             1, 3, 5, 9, 14 or 21; four tables for stiffness):
//               E[t][ks][lane] = T_t(q, k),  q = 16 qt + lane % 16, k = 4 ks + lane / 16
//               C[t][mt][r][lane] = T_t(q, i), i = 16 mt + lane % 16,
//                                  q = 16 qt + row(lane / 16, r)
//               W[64]          = w_q, q = 16 qt + j (j < 16), zero padding
//             with T_0 = phi_k (values) and T_{1+s} = d_s phi_k (stiffness),
//             row(kb, r) the output row of the matrix-core instruction
struct FormLayout {
  int d, nd, ndt, n_phi, n_q, prec, form, has_coeff;
  int kstep, kpl, n_q_pad, k_pad, nks, mt;
  int elt_bytes;  // bytes per operand element in afrag
  int tab_bytes;  // weighted table: 2 (half, FP16 mode), 4 (float) or 8 (double, FP64 mode)
  int vtab_bytes; // value table for the coefficient: 8 unless FP16/BF16 storage
  size_t off_afrag, off_afrag_lo, off_wtab, off_vtab, off_ptab, off_wq, total;
  int box;  // hexahedron: per-point |det J| (quadrature points at off_ptab)
  int act_nt, act_nks, act_mt, act_nqt;  // act_nt == 0: no action tables
  size_t act_chunk, off_act;
};

struct FormHeader {
  int32_t status;
  int32_t magic;
  int32_t d, nd, n_phi, n_q, prec, form;
  int32_t geom, pad;  // geometry precision (FE_GEOM_*)
  double max_wb;    // max |w_q B_t(q, j)|
  double lebesgue;  // max_q sum_k |phi_k(X_q)|
  double b_scale;   // exact power of two applied to the B^T operand (FP16/BF16 modes)
  double w_scale;   // exact power of two applied to the weighted table (FP16 mode)
  double max_w;     // max_q w_q
};

constexpr int32_t FORM_MAGIC = 0x46453335;  // "FE35"
constexpr size_t HEADER_BYTES = 256;

fe_status compute_layout(const fe_form_desc *f, FormLayout *L);

// Slot of the B^T fragment (16 rows x one K-step) of row tile mt, derivative
// slab s and quadrature chunk qc: chunk-major, so that the fragments of one
// chunk are contiguous.
constexpr size_t frag_slot(int mt, int s, int qc, int n_mt, int ndt) {
  return ((size_t)qc * ndt + s) * n_mt + mt;
}
fe_status check_form(const fe_form_desc *f);

// ---- cell kernel launchers, one per precision (fe_cell_<prec>.hip) ----
struct CellLaunch {
  const FormLayout *L;
  const unsigned char *form_buf;  // device
  int32_t *status;                // device status word (inside form_buf)
  int64_t n_cells;
  const double *coords;
  const int32_t *dofmap;
  int64_t n_dofs;
  const double *coeff;
  void *A_local;
  void *stream;
  int tile = -1;  // tile variant (see launch_cell_impl), < 0: default
};
// tiles 0..7: the batched cell kernel (variant + 4 occ), bitwise identical
// to each other; tile 8: the whole-cell kernel (FP16 forms it is compiled
// for, no coefficient), same precision, its own rounding order; tile 9: the
// vector-ALU kernel of the smallest FP16 mass forms (fe_smallcell.h), the
// same H, its own summation order
constexpr int CELL_TILES = 10;
constexpr int CELL_TILE_WHOLE = 8;
constexpr int CELL_TILE_SMALL = 9;
fe_status launch_cell_fp64(const CellLaunch &a);
fe_status launch_cell_fp32(const CellLaunch &a);
fe_status launch_cell_fp16(const CellLaunch &a);
fe_status launch_cell_bf16(const CellLaunch &a);
fe_status launch_cell_split(const CellLaunch &a);
fe_status launch_cell(const CellLaunch &a);
fe_status launch_small_fp16(const CellLaunch &a);  // FE_EUNSUPPORTED unless the form is one of its own

// ---- whole-cell kernel (one wave per cell, FP16), see fe_cellwise.h ----
struct CellwiseLaunch {
  const FormLayout *L;
  const unsigned char *form_buf;
  int32_t *status;
  int64_t n_cells;
  const double *coords;
  const int32_t *dofmap;
  int64_t n_dofs;
  const double *coeff;  // nodal coefficient or null
  float *zpt, *zmax;    // workspace: the coefficient at the points [n_cells][n_q_pad], its max per cell
  void *rec;            // workspace: the cell factors of a coefficient form, 32 bytes per cell
  float *A_local;       // [n_cells][n_phi][n_phi]
  void *stream;
};
// Forms the whole-cell kernel is compiled for: FP16 storage, tetrahedra,
// the Poisson form with 6 row tiles (P6) or the mass form with 4, 6 or 8
// (P5..P7), n_phi a multiple of four, or with 11 (P8); a coefficient only
// with the Poisson form.
bool cellwise_eligible(const FormLayout &L);
fe_status launch_cellwise_fp16(const CellwiseLaunch &c);

// ---- fused (row-ownership) numeric path, see fe_fused.h ----
constexpr int FUSED_SPAN = 1024;    // CSR entries per task (LDS row buffer of one wave)
// Hexahedral forms: rows of up to (2p+1)^3 entries (729 at Q4), so tasks of
// 1024 entries would hold one or two rows and fill half a tile; with half
// tables (FP16) their tasks hold up to 2048 and 8 waves still fit.
constexpr int FUSED_SPAN_BOX = 2048;
constexpr int FUSED_TILE_MAX = 4;   // tiles per task: one lane record per lane of a wave

struct FusedTask {
  int32_t r0;      // first row
  int32_t pre;     // byte t: pairs in the tiles before tile t of the task
  int32_t t0, nt;  // tiles [t0, t0 + nt)
  int64_t base;    // row_ptr[r0]: first CSR entry of the task
  int32_t span;    // row_ptr[r1] - row_ptr[r0]
  int32_t p0;      // schedule index of the task's first (cell, j) pair; the
                   // pairs of a tile fill its first lanes
};

struct FusedLane {
  int32_t cell;     // < 0: idle lane
  uint16_t rowoff;  // offset of the row inside the task's CSR span
  uint8_t j;        // local index of the row's dof in the cell
  uint8_t round;    // low 4 bits: earlier lanes of the tile holding the same
                    // row (15: idle lane); high 4 bits: the tile's last round
};

// Per-cell, per-form factors of H from the geometry pass: the symmetric
// scaled geometry tensor sigma_K G (G00 G01 G02 G11 G12 G22; mass: sigma_K
// |det J| in g[0]) in the arithmetic type of H, and the exact inverse of the
// two power-of-two scales.  NaN factors mark a degenerate cell.
template <class T>
struct FormGeo {
  T g[6];
  T inv;
  T pad;
};

struct FusedLaunch {
  // one pass over the schedule computes one form, or two forms of one
  // precision one after the other per task (the schedule-order ranks, lane
  // records and task records are then read from HBM once)
  int nforms;
  const FormLayout *L[2];
  const unsigned char *form_buf[2];
  void *geo[2];           // workspace: n_cells FormGeo records per form
  void *zpt[2];           // hexahedra: per-point factors [n_cells][n_q_pad], else NULL
  void *values[2];
  const double *coords;   // device [n_cells][d+1][d]
  int64_t n_cells;
  // geometry pass: when geo_forms > 0 this launch first writes the records
  // of geo_forms forms of this precision
  int geo_forms;
  bool run_fused;         // false: geometry pass only
  const unsigned char *geo_bufs[4];  // their form buffers (header, status word)
  int geo_nd[4];
  void *geo_out[4];
  void *geo_zpt[4];                  // hexahedra: their per-point factors
  const FormLayout *geo_L[4];
  const FusedTask *tasks;
  int64_t ntasks;         // tasks of the schedule (from the FILL phase)
  const FusedLane *lanes;
  const uint16_t *srank;  // [pairs][rstride]: LDS byte offsets, see fe_fused.h
  int rstride;
  int span;               // the schedule's task span (assembly_span)
  void *stream;
};

// LDS of the fused kernel with nw waves per workgroup over nforms forms: per
// form the weighted table (always staged: it is read per lane with 16
// different rows per K-slot) and the B^T fragments if staged, and one row
// buffer (plus a private slot per lane) per wave.
inline int fused_span(const FormLayout &L) {
  return (L.box && L.prec == FE_FP16_ACC32) ? FUSED_SPAN_BOX : FUSED_SPAN;
}
// the span of an assembly's schedule: the longer one only when every form
// takes it (a form's LDS estimate with its own span is then exact, else an
// upper bound)
inline int assembly_span(const FormLayout *L, int n) {
  for (int f = 0; f < n; ++f)
    if (fused_span(L[f]) != FUSED_SPAN_BOX) return FUSED_SPAN;
  return FUSED_SPAN_BOX;
}

inline size_t fused_lds(const FormLayout *const *L, int nforms, int nw, bool with_frags) {
  const size_t real = (L[0]->prec == FE_FP64) ? 8 : 4;
  size_t bytes = (size_t)nw * (fused_span(*L[0]) + 64) * real;
  for (int f = 0; f < nforms; ++f) {
    const FormLayout &F = *L[f];
    const size_t frag = (F.elt_bytes == 2) ? 16 : F.elt_bytes;
    if (with_frags)
      bytes += (size_t)F.mt * F.nks * 64 * frag * (F.prec == FE_SPLITFP16_ACC32 ? 2 : 1);
    const size_t tab = F.tab_bytes;
    bytes += (size_t)F.n_phi * (F.ndt * F.n_q_pad + 16 / tab) * tab;
  }
  return bytes;
}
constexpr size_t FUSED_LDS_BUDGET = 156 * 1024;
bool fused_eligible(const FormLayout &L);

// Can two forms share one fused pass: same precision and degree, one mass
// and one stiffness form with at most 4 row tiles, and both forms' tables
// next to the row buffers of at least 8 waves?
inline bool fused_pair_fits(const FormLayout *const *L) {
  return L[0]->n_phi == L[1]->n_phi && L[0]->prec == L[1]->prec && L[0]->mt <= 4 &&
         L[0]->ndt != L[1]->ndt && fused_lds(L, 2, 8, true) <= FUSED_LDS_BUDGET;
}
fe_status launch_fused_fp64(const FusedLaunch &a);
fe_status launch_fused_fp32(const FusedLaunch &a);
fe_status launch_fused_fp16(const FusedLaunch &a);
fe_status launch_fused_bf16(const FusedLaunch &a);
fe_status launch_fused_split(const FusedLaunch &a);

// ---- vector assembly plan (fe_vector_plan) and actions (fe_action.hip) ----
struct VecPlanHeader {
  int32_t status;
  int32_t magic;
  int64_t n_cells, n_dofs;
  int32_t n_phi, pad;
  int64_t max_deg;
};
constexpr int32_t VPLAN_MAGIC = 0x46455650;  // "FEVP"

// dof -> (cell, i) adjacency, entries cell * 2^ADJ_BITS + i ascending per dof
struct VecPlanLayout {
  size_t off_adj_ptr, off_cursor, off_adj, off_scan, scan_blocks, total;
};
VecPlanLayout vec_plan_layout(int64_t n_cells, int n_phi, int64_t n_dofs);

struct ActionLaunch {
  const FormLayout *L;
  const unsigned char *form_buf;
  int32_t *status;
  int64_t n_cells, n_dofs;
  const double *coords;
  const int32_t *dofmap;
  const double *coeff;  // NULL without a coefficient
  const void *x0;       // the FE function acted on
  const void *x1;       // second function of the coefficient adjoint, or NULL
  void *out0;           // local vectors [n_cells][n_phi]: action on x0
  void *out1;           // local coefficient adjoint [n_cells][n_phi] (x1 given)
  int geom;             // geometry precision (FE_GEOM_*)
  void *stream;
};
fe_status launch_action_fp32(const ActionLaunch &a);
fe_status launch_action_fp64(const ActionLaunch &a);

// Launch facts of one kernel on the current device, queried from the runtime
// once per (kernel, device, block size, LDS bytes) and cached: the compute
// unit count and the workgroups per compute unit.  The kernel's dynamic LDS
// limit is raised (once per kernel and device) to the largest size asked.
struct LaunchInfo {
  int ncu;     // compute units
  int per_cu;  // resident workgroups per compute unit (0: does not fit)
};
fe_status launch_info(const void *kern, int threads, size_t smem, LaunchInfo *out);

// Matrix-core tile choice: MT = ceil(n_phi / 16) row tiles of B^T and JC
// columns j per wave per pass (4 waves per workgroup).
void tile_choice(int n_phi, int regmul, int *mt, int *jc);

}  // namespace fe
