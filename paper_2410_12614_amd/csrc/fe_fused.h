// Fused cell kernels + CSR assembly with row ownership.
//
// Global assembly A^g = L D L^T (Section 3.3) sums, for every CSR row g, the
// rows A_K(i, :) of the cells K with dof(K, i) = g.  Here every wave owns a
// contiguous range of CSR rows ("task", at most FUSED_SPAN stored entries),
// keeps those rows in LDS, computes exactly the local rows they need and
// writes them out once, coalesced: no local matrix ever reaches HBM and no
// entry is written twice.
//
// A local row A_K(j, :) equals the column A_K(:, j) of the symmetric mass and
// Poisson forms, and a column is one matrix-core output column: with the
// left operand B^T shared by all cells, the 16 lanes of a tile may hold 16
// arbitrary (cell, j) pairs,
//
//     [A_{c_n}(i, j_n)]_{i, n} = sum_k B^T(i, k) H_{c_n}(k, j_n),
//
// so the owner computes each needed (cell, j) column once; over all owners
// every (cell, j) pair is computed exactly once (no redundant work).
//
// Determinism: a task's pairs are taken in the order of the sorted
// adjacency lists (cell ascending); lanes of one tile holding the same row
// add in rounds, in that same order.  Every CSR entry is therefore summed in
// the fixed order cell ascending, exactly as by the row gather.
//
// Latency: the per-cell factors of H come from a geometry pass (FormGeo
// records); the task record, lane records and factors of a wave's next task
// are loaded while the current task computes.  The lane records of a task
// sit one per lane and reach the lanes of a tile by cross-lane permutes.
// Two forms of one precision (mass and stiffness) can share one pass: each
// task then computes and writes the first form's rows, then the second's,
// and the schedule is read from HBM once.
#pragma once

#include <type_traits>

#include "fe_cell_kernel.h"

namespace fe {

// One form of a fused pass.
struct FusedForm {
  const unsigned char *afrag, *afrag_lo;
  const void *wtab;
  const void *geo;        // FormGeo<T>[n_cells]
  const void *zpt;        // hexahedra: per-point factors [n_cells][n_q_pad] (type of H)
  void *values;
  int n_q_pad, nks;
};

struct FusedArgs {
  FusedForm f[2];
  const FusedTask *tasks;
  int ntasks;
  const FusedLane *lanes;
  const uint16_t *srank;  // [pairs][rstride], schedule order: LDS byte offsets of a lane's outputs
                          // (lane order, four per row tile; entries past rstride are padding)
  int n_phi, rstride;
  int span;               // CSR entries of a task's row buffer (FUSED_SPAN or FUSED_SPAN_BOX)
};

// Geometry pass: FP64 geometry of every cell (Section 4.2), once, and the
// factors of H of up to four forms of one precision, with the arithmetic of
// the cell kernel.
struct GeoTargets {
  int nforms;
  int nd[4];
  const FormHeader *hdr[4];
  void *out[4];
  int32_t *status[4];
};

template <class P>
__global__ __launch_bounds__(256) void k_form_geo(const double *coords, int64_t n_cells, int d,
                                                   GeoTargets g) {
  typedef typename P::real T;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  double G[3][3], adet;
  // one geometry per cell for all forms: those share the mode of the first
  const bool ok = cell_geometry_mode(g.hdr[0]->geom, d, coords + c * (d + 1) * d, G, adet);
  for (int f = 0; f < g.nforms; ++f) {
    typename P::hreal Gp[3][3];
    T inv;
    cell_factors<P>(g.hdr[f], g.nd[f], true, ok, G, adet, 1.0, Gp, inv);
    FormGeo<T> r;
    r.g[0] = Gp[0][0];
    r.g[1] = Gp[0][1];
    r.g[2] = Gp[0][2];
    r.g[3] = Gp[1][1];
    r.g[4] = Gp[1][2];
    r.g[5] = Gp[2][2];
    r.inv = inv;
    r.pad = 0;
    ((FormGeo<T> *)g.out[f])[c] = r;
    if (!ok) atomicOr(g.status[f], STATUS_DEGENERATE);
  }
}

// Factors of a hexahedral mass form, one thread per cell: |det J(X_q)| of the
// trilinear map at every quadrature point (FP64, then in the type the cell
// kernel evaluates per-point factors in), normalised by the exact power of
// two 2^-e that brings their maximum into [1, 2), stored in the type of H
// ([n_cells][n_q_pad], zero padding); the record holds the scaled geometry
// factor sigma_K and the exact inverse of all scales times 2^e.  Every value
// is rounded as in the cell kernel, so that both assembly paths give the
// same bits.
template <class P>
__global__ __launch_bounds__(256) void k_box_geo(const double *coords, int64_t n_cells, int n_q,
                                                 int n_q_pad, const double *ptab,
                                                 const FormHeader *hdr, FormGeo<typename P::real> *out,
                                                 typename P::hreal *zpt, int32_t *status) {
  typedef typename P::real T;
  typedef typename P::hreal HT;
  typedef typename P::zreal Z;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  double x[24];
  for (int e = 0; e < 24; ++e) x[e] = coords[c * 24 + e];
  double zmax = 0.0;
  bool ok = true;
  for (int q = 0; q < n_q; ++q) {
    const double dj = box_det(x, ptab + 3 * q);
    ok = ok && dj != 0.0 && isfinite(dj);
    zmax = fmax(zmax, fabs((double)(Z)fabs(dj)));
  }
  int ez = 0;
  if (ok && zmax > 0.0 && isfinite(zmax)) {
    ez = ilogb(zmax);
    zmax = ldexp(zmax, -ez);
  }
  const T zs = (T)ldexp(1.0, -ez);
  HT *zr = zpt + c * n_q_pad;
  for (int q = 0; q < n_q_pad; ++q) {
    T v = 0;
    if (q < n_q) v = ok ? (T)(Z)fabs(box_det(x, ptab + 3 * q)) * zs : (T)NAN;
    zr[q] = (HT)v;
  }
  double G[3][3] = {{1, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  HT Gp[3][3];
  T inv;
  cell_factors<P>(hdr, 1, true, ok, G, 1.0, ok ? zmax : 1.0, Gp, inv);
  FormGeo<T> r;
  r.g[0] = Gp[0][0];
  r.g[1] = r.g[2] = r.g[3] = r.g[4] = r.g[5] = 0;
  r.inv = (T)ldexp((double)inv, ez);
  r.pad = 0;
  out[c] = r;
  if (!ok) atomicOr(status, STATUS_DEGENERATE);
}

__device__ __forceinline__ int lane_word1(const FusedLane &l) {
  return (int)l.rowoff | ((int)l.j << 16) | ((int)l.round << 24);
}

template <class T>
__device__ __forceinline__ T shfl_t(T v, int src) {
  if constexpr (sizeof(T) == 8) {
    const int2 w = *reinterpret_cast<const int2 *>(&v);
    int2 r;
    r.x = __shfl(w.x, src);
    r.y = __shfl(w.y, src);
    return *reinterpret_cast<const T *>(&r);
  } else {
    return __shfl(v, src);
  }
}

// LDS copy of one form's tables.  The weighted table holds one row per j
// with (chunk qc, slab t, K-slot entries) in the order the K loop reads
// them, so that a lane's reads are one base plus constant offsets.  Rows are
// padded by 16 bytes: the 16 lanes of a K-slot read 16 different rows j at
// the same offset, which would fall into the same LDS banks with a
// power-of-two row stride.
template <class P>
struct FormLds {
  const unsigned char *af, *afl;
  const typename P::hreal *wt;
  int jstride;
};

template <class P, int MT, int NDT, bool STAGE_A, int NW>
__device__ __forceinline__ unsigned char *stage_form(unsigned char *base, const FusedForm &F,
                                                     int nphi, int tid, FormLds<P> &out) {
  typedef typename P::hreal HT;
  typedef typename P::frag FRAG;
  const size_t frag_bytes = STAGE_A ? (size_t)MT * F.nks * 64 * sizeof(FRAG) : 0;
  unsigned char *s_af = base;
  unsigned char *s_afl = base + frag_bytes;
  HT *s_wt = (HT *)(base + frag_bytes * (P::SPLIT ? 2 : 1));
  constexpr int WPAD = 16 / sizeof(HT);
  const int jstride = NDT * F.n_q_pad + WPAD;
  if constexpr (STAGE_A) {
    const size_t n16 = frag_bytes / 16;
    for (size_t t = tid; t < n16; t += NW * 64) ((uint4 *)s_af)[t] = ((const uint4 *)F.afrag)[t];
    if constexpr (P::SPLIT)
      for (size_t t = tid; t < n16; t += NW * 64) ((uint4 *)s_afl)[t] = ((const uint4 *)F.afrag_lo)[t];
  }
  {
    // global table [t][j][n_q_pad], copied by 16-byte pieces (one piece never
    // straddles two K-steps: a K-step is 16, 32 or 128 bytes)
    constexpr int E = 16 / sizeof(HT);
    const int per_row = F.n_q_pad / E;
    const int nrows = NDT * nphi;
    for (int u = tid; u < nrows * per_row; u += NW * 64) {
      const int row = u / per_row, q = (u - row * per_row) * E;
      const int t = row / nphi, j = row - t * nphi;
      const int qc = q / P::KSTEP, qq = q - qc * P::KSTEP;
      *(uint4 *)(s_wt + (size_t)j * jstride + (qc * NDT + t) * P::KSTEP + qq) =
          ((const uint4 *)F.wtab)[u];
    }
  }
  out.af = STAGE_A ? s_af : F.afrag;
  out.afl = STAGE_A ? s_afl : F.afrag_lo;
  out.wt = s_wt;
  out.jstride = jstride;
  return (unsigned char *)(s_wt + (size_t)nphi * jstride);
}

// Lane record and factors of one tile column, handed over by cross-lane
// permutes from the lane holding slot src of the task.
template <class T>
struct Column {
  int cell, jv, rnd, maxr;
};

// Factors of H of TT tile columns (slots src[u]), from the lanes holding
// the task's records: the scaled geometry tensor (of the half type when H is
// formed in half: exact) and the exact inverse scale.
template <class P, int NDT, int TT>
__device__ __forceinline__ void tile_factors(const FormGeo<typename P::real> &cg, const int *src,
                                             typename P::hreal (&Gs)[TT][3][3],
                                             typename P::real (&inv)[TT]) {
  typedef typename P::hreal HT;
#pragma unroll
  for (int u = 0; u < TT; ++u) {
    const HT g0 = (HT)shfl_t(cg.g[0], src[u]);
    HT g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
    if constexpr (NDT > 1) {
      g1 = (HT)shfl_t(cg.g[1], src[u]);
      g2 = (HT)shfl_t(cg.g[2], src[u]);
      g3 = (HT)shfl_t(cg.g[3], src[u]);
      g4 = (HT)shfl_t(cg.g[4], src[u]);
      g5 = (HT)shfl_t(cg.g[5], src[u]);
    }
    Gs[u][0][0] = g0; Gs[u][0][1] = g1; Gs[u][0][2] = g2;
    Gs[u][1][0] = g1; Gs[u][1][1] = g3; Gs[u][1][2] = g4;
    Gs[u][2][0] = g2; Gs[u][2][1] = g4; Gs[u][2][2] = g5;
    inv[u] = shfl_t(cg.inv, src[u]);
  }
}

// LDS byte offsets (in units of the row-buffer element) of this lane's
// outputs inside the row buffer, in lane order (four per row tile: one
// 8-byte load).  Padding rows point at the lane's private slot.
template <class T, int MT, int TT>
__device__ __forceinline__ void tile_addr(const uint16_t *const *rk, int rstride, int span, int lane,
                                          int kb, int (&addr)[TT][MT][4]) {
  const int dummy = span * (int)sizeof(T) + lane * (int)sizeof(T);
#pragma unroll
  for (int u = 0; u < TT; ++u)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      // entries past the stored width are padding rows
      uint2 w = {(unsigned)(dummy | dummy << 16), (unsigned)(dummy | dummy << 16)};
      if (mt * 16 + 4 * kb < rstride) w = *(const uint2 *)(rk[u] + mt * 16);
      addr[u][mt][0] = (int)(w.x & 0xffff);
      addr[u][mt][1] = (int)(w.x >> 16);
      addr[u][mt][2] = (int)(w.y & 0xffff);
      addr[u][mt][3] = (int)(w.y >> 16);
    }
}

// Contraction of TT tiles of one form: H formed per K-slice in registers
// from the staged weighted table (rows jv[u]), against the staged B^T
// fragments (every fragment read serves all TT tiles).  K = (s, q) is
// walked q-chunk outer, s inner, as in the cell kernel.
template <class P, int MT, int NDT, bool STAGE_A, int TT, bool PZ = false>
__device__ __forceinline__ void tile_contract(const FormLds<P> &S, const FusedForm &F,
                                              const typename P::hreal (&Gs)[TT][3][3],
                                              const int *jv, const int *zc, int lane, int kb,
                                              typename P::acc (&acc)[TT][MT],
                                              typename P::acc (&acc2)[P::SPLIT ? TT : 1][P::SPLIT ? MT : 1]) {
  typedef typename P::real T;
  typedef typename P::hreal HT;
  typedef typename P::acc ACC;
  typedef typename P::frag FRAG;
  constexpr int KPL = P::KPL;
  const int nqc = F.n_q_pad / P::KSTEP;
#pragma unroll
  for (int u = 0; u < TT; ++u)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      acc[u][mt] = ACC{0, 0, 0, 0};
      if constexpr (P::SPLIT) acc2[u][mt] = ACC{0, 0, 0, 0};
    }
  // geometry factors of H in both halves of a register (half path)
  half2_t g2[TT][NDT][NDT];
#pragma unroll
  for (int u = 0; u < TT; ++u)
#pragma unroll
    for (int s = 0; s < NDT; ++s)
#pragma unroll
      for (int t = 0; t < NDT; ++t) {
        if constexpr (P::H16) g2[u][s][t] = half2_t{(_Float16)Gs[u][s][t], (_Float16)Gs[u][s][t]};
        else g2[u][s][t] = half2_t{0, 0};
      }
  const HT *wcol[TT];
#pragma unroll
  for (int u = 0; u < TT; ++u) wcol[u] = S.wt + (size_t)jv[u] * S.jstride + kb * KPL;
  // hexahedra: the per-point factors of the tile column's cell, at this
  // lane's K entries
  const HT *zrow[TT];
#pragma unroll
  for (int u = 0; u < TT; ++u)
    zrow[u] = PZ ? (const HT *)F.zpt + (size_t)zc[u] * F.n_q_pad + kb * KPL : nullptr;
  // (a padded rule holds at least one chunk: a loop entered once at least
  // keeps the compiler from clearing the accumulators twice)
  int qc = 0;
  do {
    if constexpr (P::H16) {
      // the chunk's table reads first, then per s its fragments, H and the
      // contraction
      half8_t wv[TT][NDT];
#pragma unroll
      for (int u = 0; u < TT; ++u)
#pragma unroll
        for (int t = 0; t < NDT; ++t)
          wv[u][t] = *(const half8_t *)(wcol[u] + (qc * NDT + t) * P::KSTEP);
#pragma unroll
      for (int s = 0; s < NDT; ++s) {
        FRAG af[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const size_t fi = frag_slot(mt, s, qc, MT, NDT) * 64 + lane;
          if constexpr (STAGE_A) af[mt] = lds_frag<P>(S.af, fi);
          else af[mt] = P::load(S.af, fi);
        }
#pragma unroll
        for (int u = 0; u < TT; ++u) {
          half8_t hf = form_h16<NDT>(g2[u][s], wv[u]);
          if constexpr (PZ) hf = hf * *(const half8_t *)(zrow[u] + qc * P::KSTEP);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[u][mt] = P::mma(af[mt], hf, acc[u][mt]);
        }
      }
    } else {
      T wv[TT][NDT][KPL];
#pragma unroll
      for (int u = 0; u < TT; ++u)
#pragma unroll
        for (int t = 0; t < NDT; ++t) load_w<T, KPL>(wcol[u] + (qc * NDT + t) * P::KSTEP, wv[u][t]);
#pragma unroll
      for (int s = 0; s < NDT; ++s) {
        FRAG af[MT], al[P::SPLIT ? MT : 1];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const size_t fi = frag_slot(mt, s, qc, MT, NDT) * 64 + lane;
          if constexpr (STAGE_A) {
            af[mt] = lds_frag<P>(S.af, fi);
            if constexpr (P::SPLIT) al[mt] = lds_frag<P>(S.afl, fi);
          } else {
            af[mt] = P::load(S.af, fi);
            if constexpr (P::SPLIT) al[mt] = P::load(S.afl, fi);
          }
        }
#pragma unroll
        for (int u = 0; u < TT; ++u) {
          T h[KPL];
          form_h<T, NDT, KPL>(Gs[u][s], wv[u], h);
          if constexpr (PZ) {
            T zz[KPL];
            load_w<T, KPL>(zrow[u] + qc * P::KSTEP, zz);
#pragma unroll
            for (int e = 0; e < KPL; ++e) h[e] *= zz[e];
          }
          if constexpr (P::SPLIT) {
            FRAG hh, hl;
            P::pack2(h, hh, hl);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              acc[u][mt] = P::mma(af[mt], hh, acc[u][mt]);
              acc2[u][mt] = P::mma(af[mt], hl, acc2[u][mt]);
              acc2[u][mt] = P::mma(al[mt], hh, acc2[u][mt]);
            }
          } else {
            const FRAG hf = P::pack(h);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[u][mt] = P::mma(af[mt], hf, acc[u][mt]);
          }
        }
      }
    }
  } while (++qc < nqc);
}

// The tile's results of one accumulator set, unscaled: val = acc (+ 2^-11
// acc2 for the split pair) times the exact inverse scale.
template <class P, int MT, int TT>
__device__ __forceinline__ void tile_values(const typename P::acc (&acc)[TT][MT],
                                            const typename P::acc (&acc2)[P::SPLIT ? TT : 1][P::SPLIT ? MT : 1],
                                            int u, typename P::real inv,
                                            typename P::real (&val)[MT][4]) {
  typedef typename P::real T;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T v = acc[u][mt][q];
      if constexpr (P::SPLIT) v += acc2[u][mt][q] * (T)(1.0 / 2048.0);
      val[mt][q] = v * inv;
    }
}

// TT tiles (1 or 2) of one form: factors, output offsets, contraction, then
// the scatter into the row buffer, tile after tile, one round per repeated
// row; within a round every lane adds to a different entry (padding rows
// update the lane's private slot instead: no branch per entry).  `after_k`
// runs between the contraction and the scatter (used to issue the next
// task's loads).
template <class P, int MT, int NDT, bool STAGE_A, int TT, bool PZ, class AfterK>
__device__ __forceinline__ void fused_tiles(const FormLds<P> &S, const FusedForm &F,
                                            const FormGeo<typename P::real> &cg, const int *src,
                                            const Column<typename P::real> *col,
                                            const uint16_t *const *rk, int rstride, int span,
                                            int lane, int kb, typename P::real *rowbuf,
                                            AfterK after_k) {
  typedef typename P::real T;
  typename P::hreal Gs[TT][3][3];
  T inv[TT];
  tile_factors<P, NDT, TT>(cg, src, Gs, inv);
  int addr[TT][MT][4];
  tile_addr<T, MT, TT>(rk, rstride, span, lane, kb, addr);
  int jv[TT];
#pragma unroll
  for (int u = 0; u < TT; ++u) jv[u] = col[u].jv;
  int zc[TT];
#pragma unroll
  for (int u = 0; u < TT; ++u) zc[u] = col[u].cell < 0 ? 0 : col[u].cell;
  typename P::acc acc[TT][MT];
  typename P::acc acc2[P::SPLIT ? TT : 1][P::SPLIT ? MT : 1];
  tile_contract<P, MT, NDT, STAGE_A, TT, PZ>(S, F, Gs, jv, zc, lane, kb, acc, acc2);

  after_k();

  unsigned char *rb = (unsigned char *)rowbuf;
#pragma unroll
  for (int u = 0; u < TT; ++u) {
    T val[MT][4];
    tile_values<P, MT, TT>(acc, acc2, u, inv[u], val);
    for (int r = 0; r <= col[u].maxr; ++r) {
      if (col[u].rnd == r) {
        // read all, then write all: a lane's entries are distinct and the
        // lanes of one round hold distinct rows (the buffer starts at zero)
        T old[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int q = 0; q < 4; ++q) old[mt][q] = *(const T *)(rb + addr[u][mt][q]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int q = 0; q < 4; ++q) *(T *)(rb + addr[u][mt][q]) = old[mt][q] + val[mt][q];
      }
    }
  }
}

// TT tiles (1 or 2) of two forms sharing one row buffer of value pairs
// (form 0, form 1) per entry: all contractions (the tiles share every
// fragment read), then, tile after tile, one scatter of the pairs, so the
// scatter's LDS operations serve both forms.  The offsets of the
// schedule-order ranks count single values and are doubled here.
template <class P, int MT, int NDT0, int NDT1, bool STAGE_A, int TT, class AfterK>
__device__ __forceinline__ void fused_tile_pair(const FormLds<P> &S0, const FormLds<P> &S1,
                                                const FusedForm &F0, const FusedForm &F1,
                                                const FormGeo<typename P::real> &cg0,
                                                const FormGeo<typename P::real> &cg1,
                                                const int *src, const Column<typename P::real> *col,
                                                const uint16_t *const *rk, int rstride, int span,
                                                int lane, int kb, typename P::real *rowbuf,
                                                AfterK after_k) {
  typedef typename P::real T;
  typedef typename P::acc ACC;
  int addr[TT][MT][4];
  tile_addr<T, MT, TT>(rk, rstride, span, lane, kb, addr);
  int jv[TT];
#pragma unroll
  for (int u = 0; u < TT; ++u) jv[u] = col[u].jv;
  T val0[TT][MT][4], val1[TT][MT][4];
  {
    typename P::hreal Gs[TT][3][3];
    T inv[TT];
    tile_factors<P, NDT0, TT>(cg0, src, Gs, inv);
    ACC acc[TT][MT];
    ACC acc2[P::SPLIT ? TT : 1][P::SPLIT ? MT : 1];
    tile_contract<P, MT, NDT0, STAGE_A, TT>(S0, F0, Gs, jv, jv, lane, kb, acc, acc2);
#pragma unroll
    for (int u = 0; u < TT; ++u) tile_values<P, MT, TT>(acc, acc2, u, inv[u], val0[u]);
  }
  {
    typename P::hreal Gs[TT][3][3];
    T inv[TT];
    tile_factors<P, NDT1, TT>(cg1, src, Gs, inv);
    ACC acc[TT][MT];
    ACC acc2[P::SPLIT ? TT : 1][P::SPLIT ? MT : 1];
    tile_contract<P, MT, NDT1, STAGE_A, TT>(S1, F1, Gs, jv, jv, lane, kb, acc, acc2);
#pragma unroll
    for (int u = 0; u < TT; ++u) tile_values<P, MT, TT>(acc, acc2, u, inv[u], val1[u]);
  }

  after_k();

  typedef typename std::conditional<sizeof(T) == 4, float2, double2>::type T2;
  unsigned char *rb = (unsigned char *)rowbuf;
#pragma unroll
  for (int u = 0; u < TT; ++u) {
    for (int r = 0; r <= col[u].maxr; ++r) {
      if (col[u].rnd == r) {
        T2 old[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int q = 0; q < 4; ++q) old[mt][q] = *(const T2 *)(rb + 2 * addr[u][mt][q]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *(T2 *)(rb + 2 * addr[u][mt][q]) =
                T2{old[mt][q].x + val0[u][mt][q], old[mt][q].y + val1[u][mt][q]};
      }
    }
  }
}

// PR: the two forms share one row buffer of value pairs and one pass over
// each task's tiles (fused_tile_pair); else each form runs its own pass over
// the tiles with its own row buffer contents.
template <class P, int MT, int NDT0, int NDT1, int NF, bool STAGE_A, int NW, int TT, bool PR,
          bool PZ = false>
__global__ __launch_bounds__(NW * 64) void fused_kernel(FusedArgs a) {
  typedef typename P::real T;
  typedef FormGeo<T> GEO;
  static_assert(!PR || NF == 2, "paired rows need two forms");
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = lane & 15, kb = lane >> 4;
  const int nphi = a.n_phi;

  FormLds<P> S0, S1;
  unsigned char *end = stage_form<P, MT, NDT0, STAGE_A, NW>(smem, a.f[0], nphi, tid, S0);
  if constexpr (NF == 2) end = stage_form<P, MT, NDT1, STAGE_A, NW>(end, a.f[1], nphi, tid, S1);
  T *rowbuf = (T *)end + (size_t)wave * (a.span + 64) * (PR ? 2 : 1);
  // the row buffer's entries start at zero; the write-back of every task
  // clears what it read
  for (int t = lane; t < a.span * (PR ? 2 : 1); t += 64) rowbuf[t] = 0;
  __syncthreads();

  const int ntasks = a.ntasks;
  const int stride = gridDim.x * NW;
  int task = blockIdx.x * NW + wave;

  // lane record (two words) and factors of slot `lane` of the wave's task
  FusedTask tk{};
  int lw0 = -1, lw1 = 0;
  GEO gg[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) gg[f] = GEO{};
  if (task < ntasks) {
    tk = a.tasks[task];
    if (lane < tk.nt * 16) {
      const FusedLane l = a.lanes[(size_t)tk.t0 * 16 + lane];
      lw0 = l.cell;
      lw1 = lane_word1(l);
    }
    if (lw0 >= 0)
#pragma unroll
      for (int f = 0; f < NF; ++f) gg[f] = ((const GEO *)a.f[f].geo)[lw0];
  }

  while (task < ntasks) {
    const int nt = tk.nt, span = tk.span, p0 = tk.p0, pre = tk.pre;
    const int64_t base = tk.base;
    const int cw0 = lw0, cw1 = lw1;
    GEO cg[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) cg[f] = gg[f];
    const int next = task + stride;
    const bool has_next = next < ntasks;
    if (has_next) tk = a.tasks[next];

#pragma unroll
    for (int f = 0; f < (PR ? 1 : NF); ++f) {
      for (int tl = 0; tl < nt;) {
        // tiles processed together: up to TT while that many remain
        const int tt = min(TT, nt - tl);
        int src[TT];
        Column<T> col[TT];
        const uint16_t *rk[TT];
#pragma unroll
        for (int u = 0; u < TT; ++u) {
          const int t = tl + (u < tt ? u : 0);
          // this lane's column: slot 16 t + n of the task
          src[u] = 16 * t + n;
          col[u].cell = __shfl(cw0, src[u]);
          const int w1 = __shfl(cw1, src[u]);
          col[u].jv = (w1 >> 16) & 0xff;
          col[u].rnd = (w1 >> 24) & 0xf;
          // the tile's last round, the same in every lane record of the tile
          col[u].maxr = __builtin_amdgcn_readfirstlane((int)((unsigned)w1 >> 28));
          const int pair = col[u].cell < 0 ? 0 : p0 + ((pre >> (8 * t)) & 0xff) + n;
          rk[u] = a.srank + (size_t)pair * a.rstride + 4 * kb;
        }
        // the next task's lane records and then its factors, behind the
        // first tiles' contraction
        if (f == 0 && tl == 0 && has_next) {
          lw0 = -1;
          lw1 = 0;
          if (lane < tk.nt * 16) {
            const FusedLane l = a.lanes[(size_t)tk.t0 * 16 + lane];
            lw0 = l.cell;
            lw1 = lane_word1(l);
          }
        }
        // (the factors are held only from the last form's first tiles on)
        auto after_k = [&]() {
          if ((PR || f == NF - 1) && tl == 0 && has_next) {
#pragma unroll
            for (int e = 0; e < NF; ++e) gg[e] = GEO{};
            if (lw0 >= 0)
#pragma unroll
              for (int e = 0; e < NF; ++e) gg[e] = ((const GEO *)a.f[e].geo)[lw0];
          }
        };
        if constexpr (PR) {
          if (tt == 3) {
            if constexpr (TT == 3)
              fused_tile_pair<P, MT, NDT0, NDT1, STAGE_A, 3>(S0, S1, a.f[0], a.f[1], cg[0],
                                                             cg[NF - 1], src, col, rk, a.rstride, a.span,
                                                             lane, kb, rowbuf, after_k);
          } else if (tt == 2) {
            if constexpr (TT >= 2)
              fused_tile_pair<P, MT, NDT0, NDT1, STAGE_A, 2>(S0, S1, a.f[0], a.f[1], cg[0],
                                                             cg[NF - 1], src, col, rk, a.rstride, a.span,
                                                             lane, kb, rowbuf, after_k);
          } else {
            fused_tile_pair<P, MT, NDT0, NDT1, STAGE_A, 1>(S0, S1, a.f[0], a.f[1], cg[0],
                                                           cg[NF - 1], src, col, rk, a.rstride, a.span,
                                                           lane, kb, rowbuf, after_k);
          }
        } else if (tt == 2) {
          if constexpr (TT >= 2) {
            if (f == 0)
              fused_tiles<P, MT, NDT0, STAGE_A, 2, PZ>(S0, a.f[0], cg[0], src, col, rk, a.rstride, a.span,
                                                   lane, kb, rowbuf, after_k);
            else if constexpr (NF == 2)
              fused_tiles<P, MT, NDT1, STAGE_A, 2, false>(S1, a.f[1], cg[NF - 1], src, col, rk,
                                                   a.rstride, a.span, lane, kb, rowbuf, after_k);
          }
        } else {
          if (f == 0)
            fused_tiles<P, MT, NDT0, STAGE_A, 1, PZ>(S0, a.f[0], cg[0], src, col, rk, a.rstride, a.span, lane,
                                                 kb, rowbuf, after_k);
          else if constexpr (NF == 2)
            fused_tiles<P, MT, NDT1, STAGE_A, 1, false>(S1, a.f[1], cg[NF - 1], src, col, rk, a.rstride, a.span,
                                                 lane, kb, rowbuf, after_k);
        }
        tl += tt;
      }
      // write-back of the task's rows: single precision in groups of four
      // consecutive entries per lane (one 16-byte store each), the rest one
      // by one
      const int s4 = sizeof(T) == 4 ? (span & ~3) : 0;
      if constexpr (PR) {
        typedef typename std::conditional<sizeof(T) == 4, float2, double2>::type T2;
        T *V0 = (T *)a.f[0].values + base;
        T *V1 = (T *)a.f[NF - 1].values + base;
        if constexpr (sizeof(T) == 4) {
          for (int t = 4 * lane; t < s4; t += 256) {
            const float4 p = *(const float4 *)(rowbuf + 2 * t);
            const float4 q = *(const float4 *)(rowbuf + 2 * t + 4);
            *(float4 *)(rowbuf + 2 * t) = float4{0, 0, 0, 0};
            *(float4 *)(rowbuf + 2 * t + 4) = float4{0, 0, 0, 0};
            *(f4u_t *)(V0 + t) = f4u_t{p.x, p.z, q.x, q.z};
            *(f4u_t *)(V1 + t) = f4u_t{p.y, p.w, q.y, q.w};
          }
        }
        for (int t = s4 + lane; t < span; t += 64) {
          const T2 v = ((const T2 *)rowbuf)[t];
          ((T2 *)rowbuf)[t] = T2{0, 0};
          V0[t] = v.x;
          V1[t] = v.y;
        }
      } else {
        T *V = (T *)a.f[f].values + base;
        if constexpr (sizeof(T) == 4) {
          for (int t = 4 * lane; t < s4; t += 256) {
            const float4 p = *(const float4 *)(rowbuf + t);
            *(float4 *)(rowbuf + t) = float4{0, 0, 0, 0};
            *(f4u_t *)(V + t) = f4u_t{p.x, p.y, p.z, p.w};
          }
        }
        for (int t = s4 + lane; t < span; t += 64) {
          V[t] = rowbuf[t];
          rowbuf[t] = 0;
        }
      }
    }
    task = next;
  }
}

template <class P, int MT, int NDT0, int NDT1, int NF, bool SA, int NW, int TT, bool PR = false,
          bool PZ = false>
static fe_status launch_fused_one(const FusedArgs &k, size_t smem, hipStream_t s) {
  auto kern = fused_kernel<P, MT, NDT0, NDT1, NF, SA, NW, TT, PR, PZ>;
  LaunchInfo li;
  if (launch_info((const void *)kern, NW * 64, smem, &li) != FE_OK) return FE_EHIP;
  const int ncu = li.ncu, per_cu = li.per_cu;
  if (per_cu < 1) return FE_EUNSUPPORTED;
  const int64_t need = ((int64_t)k.ntasks + NW - 1) / NW;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)ncu * per_cu));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), smem, s, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

// Whether an instantiation of the fused kernel keeps per-lane values in
// scratch memory (register spills), as the compiled code object reports it;
// asked once per instantiation.
template <class P, int MT, int NDT0, int NDT1, int NF, bool SA, int NW, int TT, bool PR, bool PZ>
static bool fused_spills() {
  static const bool spills = [] {
    hipFuncAttributes at;
    return hipFuncGetAttributes(&at, (const void *)fused_kernel<P, MT, NDT0, NDT1, NF, SA, NW, TT, PR, PZ>) ==
               hipSuccess &&
           at.localSizeBytes > 0;
  }();
  return spills;
}

template <class P, int MT, int NDT0, int NDT1, int NF, bool PZ = false>
static fe_status launch_fused_nw(const FusedArgs &k, const FormLayout *const *L, hipStream_t s) {
  // A pair shares one row buffer of value pairs (one scatter for both
  // forms) when that fits with 8 waves, several tiles per step where their
  // accumulators fit the register file: three in half precision (a task of
  // the P4 benchmark workload mostly holds 33 to 48 columns, so one step
  // covers it and each fragment read serves three tiles: 4 % faster than two
  // per step, which was 3 % faster than one), two in FP32; the split and FP64
  // pairs spill with two and take one.  Otherwise one tile
  // per step with the most waves per workgroup that fit with the fragments
  // staged (at least 8: see fused_eligible) and hold the tile in registers
  // (16 waves get 128 registers each, 12 get 168: larger tiles spill there,
  // which cost the Q4 hexahedral pass more than half its time); there 16
  // waves with one tile per step beat 12 waves with two tiles sharing each
  // fragment read.
  if constexpr (PZ) {
    // hexahedra (single mass form): 16 waves, else 8
    if (fused_lds(L, NF, 16, true) <= FUSED_LDS_BUDGET &&
        !fused_spills<P, MT, NDT0, NDT1, NF, true, 16, 1, false, true>())
      return launch_fused_one<P, MT, NDT0, NDT1, NF, true, 16, 1, false, true>(k, fused_lds(L, NF, 16, true), s);
    if (fused_lds(L, NF, 8, true) <= FUSED_LDS_BUDGET)
      return launch_fused_one<P, MT, NDT0, NDT1, NF, true, 8, 1, false, true>(k, fused_lds(L, NF, 8, true), s);
    return FE_EUNSUPPORTED;
  }
  if constexpr (NF == 2) {
    const size_t pr = fused_lds(L, NF, 8, true) + (size_t)8 * (FUSED_SPAN + 64) * sizeof(typename P::real);
    constexpr int PTT = (P::SPLIT || sizeof(typename P::real) == 8) ? 1 : (P::H16 ? 3 : 2);
    if (pr <= FUSED_LDS_BUDGET)
      return launch_fused_one<P, MT, NDT0, NDT1, NF, true, 8, PTT, true>(k, pr, s);
  }
  if (fused_lds(L, NF, 16, true) <= FUSED_LDS_BUDGET &&
      !fused_spills<P, MT, NDT0, NDT1, NF, true, 16, 1, false, false>())
    return launch_fused_one<P, MT, NDT0, NDT1, NF, true, 16, 1>(k, fused_lds(L, NF, 16, true), s);
  if (fused_lds(L, NF, 12, true) <= FUSED_LDS_BUDGET &&
      !fused_spills<P, MT, NDT0, NDT1, NF, true, 12, 1, false, false>())
    return launch_fused_one<P, MT, NDT0, NDT1, NF, true, 12, 1>(k, fused_lds(L, NF, 12, true), s);
  if (fused_lds(L, NF, 8, true) <= FUSED_LDS_BUDGET)
    return launch_fused_one<P, MT, NDT0, NDT1, NF, true, 8, 1>(k, fused_lds(L, NF, 8, true), s);
  return FE_EUNSUPPORTED;
}

template <class P>
fe_status launch_fused_impl(const FusedLaunch &a) {
  typedef typename P::real T;
  const FormLayout *const *L = a.L;
  hipStream_t s = (hipStream_t)a.stream;
  for (int f = 0; f < a.nforms; ++f)
    if (!fused_eligible(*L[f])) return FE_EUNSUPPORTED;
  if (a.nforms == 2 && (!fused_pair_fits(L) || L[0]->box || L[1]->box)) return FE_EUNSUPPORTED;
  if (a.n_cells > 0 && a.geo_forms > 0 && L[0]->box) {
    // hexahedra: per cell |det J| at every quadrature point
    for (int f = 0; f < a.geo_forms; ++f) {
      const FormHeader *h = (const FormHeader *)a.geo_bufs[f];
      const FormLayout &G = *a.geo_L[f];
      if (!a.geo_zpt[f]) return FE_EINVAL;
      hipLaunchKernelGGL(k_box_geo<P>, dim3((unsigned)((a.n_cells + 255) / 256)), dim3(256), 0, s,
                         a.coords, a.n_cells, G.n_q, G.n_q_pad,
                         (const double *)(a.geo_bufs[f] + G.off_ptab), h,
                         (FormGeo<T> *)a.geo_out[f], (typename P::hreal *)a.geo_zpt[f],
                         (int32_t *)a.geo_bufs[f]);
    }
    if (hipGetLastError() != hipSuccess) return FE_EHIP;
  } else if (a.n_cells > 0 && a.geo_forms > 0) {
    GeoTargets g;
    g.nforms = a.geo_forms;
    for (int f = 0; f < a.geo_forms; ++f) {
      g.nd[f] = a.geo_nd[f];
      g.hdr[f] = (const FormHeader *)a.geo_bufs[f];
      g.out[f] = a.geo_out[f];
      g.status[f] = (int32_t *)a.geo_bufs[f];
    }
    hipLaunchKernelGGL(k_form_geo<P>, dim3((unsigned)((a.n_cells + 255) / 256)), dim3(256), 0, s,
                       a.coords, a.n_cells, L[0]->d, g);
    if (hipGetLastError() != hipSuccess) return FE_EHIP;
  }
  if (a.ntasks <= 0 || !a.run_fused) return FE_OK;
  if (L[0]->box && !a.zpt[0]) return FE_EINVAL;
  FusedArgs k;
  for (int f = 0; f < 2; ++f) {
    const int e = f < a.nforms ? f : 0;
    k.f[f].afrag = a.form_buf[e] + L[e]->off_afrag;
    k.f[f].afrag_lo = a.form_buf[e] + L[e]->off_afrag_lo;
    k.f[f].wtab = a.form_buf[e] + L[e]->off_wtab;
    k.f[f].geo = a.geo[e];
    k.f[f].zpt = a.zpt[e];
    k.f[f].values = a.values[e];
    k.f[f].n_q_pad = L[e]->n_q_pad;
    k.f[f].nks = L[e]->nks;
  }
  k.tasks = a.tasks;
  k.ntasks = (int)a.ntasks;
  k.lanes = a.lanes;
  k.srank = a.srank;
  k.n_phi = L[0]->n_phi;
  k.rstride = a.rstride;
  k.span = a.span;
  if (k.span < FUSED_SPAN || k.span > fused_span(*L[0])) return FE_EINVAL;
  const int mt = L[0]->mt;
  const int d0 = L[0]->ndt, d1 = a.nforms == 2 ? L[1]->ndt : 1;
#define FE_FL(M)                                                                         \
  if (mt == M) {                                                                         \
    if (a.nforms == 1) {                                                                 \
      if (L[0]->box) return launch_fused_nw<P, M, 1, 1, 1, true>(k, L, s);               \
      if (d0 == 1) return launch_fused_nw<P, M, 1, 1, 1>(k, L, s);                       \
      return launch_fused_nw<P, M, 3, 1, 1>(k, L, s);                                    \
    }                                                                                    \
    if constexpr (M <= 4) {                                                              \
      if (d0 == 1 && d1 == 3) return launch_fused_nw<P, M, 1, 3, 2>(k, L, s);            \
      if (d0 == 3 && d1 == 1) return launch_fused_nw<P, M, 3, 1, 2>(k, L, s);            \
    }                                                                                    \
    return FE_EUNSUPPORTED;                                                              \
  }
  FE_FL(1) FE_FL(2) FE_FL(3) FE_FL(4) FE_FL(6) FE_FL(8) FE_FL(11)
#undef FE_FL
  return FE_EUNSUPPORTED;
}

}  // namespace fe
