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
#pragma once

#include "fe_cell_kernel.h"

namespace fe {

struct FusedArgs {
  const unsigned char *afrag, *afrag_lo;
  const void *wtab;
  const FormHeader *hdr;
  const CellGeo *geo;
  const FusedTask *tasks;
  const int32_t *ntasks;
  const FusedLane *lanes;
  const uint16_t *rank;   // [n_cells][n_phi][n_phi]: rank of dof(K, i) in row dof(K, j) at [K][j][i]
  const int64_t *row_ptr;
  void *values;
  int n_phi, nd, n_q_pad, nks;
};

template <class P, int MT, int NDT, bool STAGE_A, bool STAGE_W>
__global__ __launch_bounds__(FUSED_WAVES * 64) void fused_kernel(FusedArgs a) {
  typedef typename P::real T;
  typedef typename P::acc ACC;
  typedef typename P::frag FRAG;
  constexpr int TT = FUSED_TT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = lane & 15, kb = lane >> 4;
  const int nphi = a.n_phi, n_q_pad = a.n_q_pad, nks = a.nks;

  // staged weighted-table rows are padded by 16 bytes: the 16 lanes of a
  // K-slot read 16 different rows j at the same offset, which would all fall
  // into the same LDS banks with an unpadded power-of-two row stride
  constexpr int WPAD = 16 / sizeof(T);
  const int wrow = n_q_pad + WPAD;
  const size_t frag_bytes = STAGE_A ? (size_t)MT * nks * 64 * sizeof(FRAG) : 0;
  const size_t wtab_bytes = STAGE_W ? (size_t)NDT * nphi * wrow * sizeof(T) : 0;
  unsigned char *s_af = smem;
  unsigned char *s_afl = smem + frag_bytes;
  T *s_wt = (T *)(smem + frag_bytes * (P::SPLIT ? 2 : 1));
  T *rowbuf = (T *)(smem + frag_bytes * (P::SPLIT ? 2 : 1) + wtab_bytes) + (size_t)wave * FUSED_SPAN;

  if constexpr (STAGE_A) {
    const size_t n16 = frag_bytes / 16;
    for (size_t t = tid; t < n16; t += FUSED_WAVES * 64) ((uint4 *)s_af)[t] = ((const uint4 *)a.afrag)[t];
    if constexpr (P::SPLIT)
      for (size_t t = tid; t < n16; t += FUSED_WAVES * 64)
        ((uint4 *)s_afl)[t] = ((const uint4 *)a.afrag_lo)[t];
  }
  if constexpr (STAGE_W) {
    const int per_row = n_q_pad * (int)sizeof(T) / 16;   // 16-byte chunks per row
    const int nrows = NDT * nphi;
    for (int t = tid; t < nrows * per_row; t += FUSED_WAVES * 64) {
      const int row = t / per_row, col = t - row * per_row;
      ((uint4 *)(s_wt + (size_t)row * wrow))[col] = ((const uint4 *)a.wtab)[(size_t)row * per_row + col];
    }
  }
  if constexpr (STAGE_A || STAGE_W) __syncthreads();
  const int ebs = ilogb(a.hdr->b_scale);

  const int ntasks = *a.ntasks;
  for (int task = blockIdx.x * FUSED_WAVES + wave; task < ntasks; task += gridDim.x * FUSED_WAVES) {
    const FusedTask tk = a.tasks[task];
    const int64_t base = tk.base;
    const int span = tk.span;
    for (int t = lane; t < span; t += 64) rowbuf[t] = 0;

    for (int t0 = 0; t0 < tk.nt; t0 += TT) {
      int cell[TT], jv[TT], roff[TT], rnd[TT];
      T Gp[TT][3][3];
      T inv[TT];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        cell[tt] = -1;
        jv[tt] = 0;
        roff[tt] = 0;
        rnd[tt] = 0;
        if (t0 + tt < tk.nt) {
          const FusedLane L = a.lanes[(size_t)(tk.t0 + t0 + tt) * 16 + n];
          cell[tt] = L.cell;
          jv[tt] = L.j;
          roff[tt] = L.rowoff;
          rnd[tt] = L.round;
        }
        double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        double sK = 1.0, adet = 0.0;
        int esK = 0;
        bool ok = true;
        if (cell[tt] >= 0) {
          const CellGeo cg = a.geo[cell[tt]];
          G[0][0] = cg.g[0]; G[0][1] = G[1][0] = cg.g[1]; G[0][2] = G[2][0] = cg.g[2];
          G[1][1] = cg.g[3]; G[1][2] = G[2][1] = cg.g[4]; G[2][2] = cg.g[5];
          adet = cg.adet;
          ok = cg.ok != 0.0;
          double gabs = adet;
          if (a.nd > 1) {
            gabs = 0.0;
            for (int s = 0; s < 3; ++s) gabs = fmax(gabs, fabs(G[s][0]) + fabs(G[s][1]) + fabs(G[s][2]));
          }
          if constexpr (P::SCALED) {
            const double bound = a.hdr->max_wb * gabs;
            if (bound > 0.0 && isfinite(bound)) {
              esK = 14 - ilogb(bound);
              sK = ldexp(1.0, esK);
            }
          }
        }
        for (int s = 0; s < 3; ++s)
          for (int t = 0; t < 3; ++t) {
            double v = (a.nd == 1) ? (s == 0 && t == 0 ? adet : 0.0) : G[s][t];
            if (cell[tt] < 0) v = 0.0;
            else if (!ok) v = NAN;
            Gp[tt][s][t] = (T)(v * sK);
          }
        // sK and the B scale are exact powers of two: invert by exponents
        inv[tt] = (T)ldexp(1.0, -esK - ebs);
      }

      // positions of this tile's outputs inside their rows, loaded before the
      // contraction so that their latency hides behind it
      int rv[TT][MT][4];
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        const uint16_t *rk = a.rank + ((size_t)(cell[tt] < 0 ? 0 : cell[tt]) * nphi + jv[tt]) * nphi;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = mt * 16 + P::row(kb, q);
            rv[tt][mt][q] = (cell[tt] >= 0 && i < nphi) ? (int)rk[i] : -1;
          }
      }

      ACC acc[MT][TT];
      ACC acc2[P::SPLIT ? MT : 1][P::SPLIT ? TT : 1];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) {
          acc[mt][tt] = ACC{0, 0, 0, 0};
          if constexpr (P::SPLIT) acc2[mt][tt] = ACC{0, 0, 0, 0};
        }
      for (int ks = 0; ks < nks; ++ks) {
        const int k0 = ks * P::KSTEP;
        const int s = k0 / n_q_pad;
        const int qb = k0 - s * n_q_pad + kb * P::KPL;
        FRAG afr[MT];
        FRAG afl[P::SPLIT ? MT : 1];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const size_t fi = ((size_t)mt * nks + ks) * 64 + lane;
          if constexpr (STAGE_A) {
            afr[mt] = lds_frag<P>(s_af, fi);
            if constexpr (P::SPLIT) afl[mt] = lds_frag<P>(s_afl, fi);
          } else {
            afr[mt] = P::load(a.afrag, fi);
            if constexpr (P::SPLIT) afl[mt] = P::load(a.afrag_lo, fi);
          }
        }
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) {
          T h[P::KPL];
#pragma unroll
          for (int e = 0; e < P::KPL; ++e) h[e] = 0;
#pragma unroll
          for (int t = 0; t < NDT; ++t) {
            const T g = (s == 0) ? Gp[tt][0][t] : ((s == 1) ? Gp[tt][1][t] : Gp[tt][2][t]);
            const T *w;
            if constexpr (STAGE_W) w = s_wt + ((size_t)t * nphi + jv[tt]) * wrow + qb;
            else w = (const T *)a.wtab + ((size_t)t * nphi + jv[tt]) * n_q_pad + qb;
            T wv[P::KPL];
            if constexpr (P::KPL == 8) {
              const float4 w0 = ((const float4 *)w)[0], w1 = ((const float4 *)w)[1];
              wv[0] = w0.x; wv[1] = w0.y; wv[2] = w0.z; wv[3] = w0.w;
              wv[4] = w1.x; wv[5] = w1.y; wv[6] = w1.z; wv[7] = w1.w;
            } else {
              wv[0] = w[0];
            }
#pragma unroll
            for (int e = 0; e < P::KPL; ++e) h[e] += g * wv[e];
          }
          if constexpr (P::SPLIT) {
            FRAG hh, hl;
            P::pack2(h, hh, hl);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              acc[mt][tt] = P::mma(afr[mt], hh, acc[mt][tt]);
              acc2[mt][tt] = P::mma(afr[mt], hl, acc2[mt][tt]);
              acc2[mt][tt] = P::mma(afl[mt], hh, acc2[mt][tt]);
            }
          } else {
            const FRAG hf = P::pack(h);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt][tt] = P::mma(afr[mt], hf, acc[mt][tt]);
          }
        }
      }

      // scatter into the owned rows, one round per repeated row
#pragma unroll
      for (int tt = 0; tt < TT; ++tt) {
        if (t0 + tt >= tk.nt) break;
        int maxr = rnd[tt];
        for (int off = 1; off < 64; off <<= 1) maxr = max(maxr, __shfl_xor(maxr, off));
        for (int r = 0; r <= maxr; ++r) {
          if (cell[tt] >= 0 && rnd[tt] == r) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                if (rv[tt][mt][q] >= 0) {
                  T v = acc[mt][tt][q];
                  if constexpr (P::SPLIT) v += acc2[mt][tt][q] * (T)(1.0 / 2048.0);
                  rowbuf[roff[tt] + rv[tt][mt][q]] += v * inv[tt];
                }
              }
          }
        }
      }
    }
    T *V = (T *)a.values + base;
    for (int t = lane; t < span; t += 64) V[t] = rowbuf[t];
  }
}

template <class P, int MT, int NDT, bool SA, bool SW>
static fe_status launch_fused_one(const FusedArgs &k, int64_t ntasks_max, size_t smem,
                                  hipStream_t s) {
  auto kern = fused_kernel<P, MT, NDT, SA, SW>;
  if (smem > 65536 && hipFuncSetAttribute((const void *)kern,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)smem) != hipSuccess)
    return FE_EHIP;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return FE_EHIP;
  const int64_t need = (ntasks_max + FUSED_WAVES - 1) / FUSED_WAVES;
  const int per_cu = smem <= 76 * 1024 ? 2 : 1;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)ncu * per_cu));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(FUSED_WAVES * 64), smem, s, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

// LDS staging of the fused kernel: the weighted table is read per lane with
// 16 different rows per K-slot, so the fused path is used only when it fits
// in LDS next to the row buffers (else the caller takes the row-gather path).
inline bool fused_staging(const FormLayout *L, bool *sa, bool *sw) {
  const size_t real = (L->prec == FE_FP64) ? 8 : 4;
  const size_t frag = (L->elt_bytes == 2) ? 16 : L->elt_bytes;
  const size_t rows_bytes = (size_t)FUSED_WAVES * FUSED_SPAN * real;
  const size_t frag_bytes =
      (size_t)L->mt * L->nks * 64 * frag * (L->prec == FE_SPLITFP16_ACC32 ? 2 : 1);
  const size_t wtab_bytes = (size_t)L->ndt * L->n_phi * (L->n_q_pad + 16 / real) * real;
  const size_t budget = 156 * 1024;
  // the table is required in LDS; the B^T fragments join it when room remains
  *sw = wtab_bytes + rows_bytes <= budget;
  *sa = *sw && frag_bytes + wtab_bytes + rows_bytes <= budget;
  return true;
}

template <class P>
fe_status launch_fused_impl(const FusedLaunch &a) {
  const FormLayout &L = *a.L;
  typedef typename P::frag FRAG;
  FusedArgs k;
  k.afrag = a.form_buf + L.off_afrag;
  k.afrag_lo = a.form_buf + L.off_afrag_lo;
  k.wtab = a.form_buf + L.off_wtab;
  k.hdr = (const FormHeader *)a.form_buf;
  k.geo = a.geo;
  k.tasks = a.tasks;
  k.ntasks = a.ntasks;
  k.lanes = a.lanes;
  k.rank = a.rank;
  k.row_ptr = a.row_ptr;
  k.values = a.values;
  k.n_phi = L.n_phi;
  k.nd = L.nd;
  k.n_q_pad = L.n_q_pad;
  k.nks = L.nks;
  const size_t rows_bytes = (size_t)FUSED_WAVES * FUSED_SPAN * sizeof(typename P::real);
  const size_t frag_bytes = (size_t)L.mt * L.nks * 64 * sizeof(FRAG) * (P::SPLIT ? 2 : 1);
  const size_t wtab_bytes =
      (size_t)L.ndt * L.n_phi * (L.n_q_pad + 16 / sizeof(typename P::real)) * sizeof(typename P::real);
  bool sa, sw;
  if (!fused_staging(a.L, &sa, &sw) || !sw) return FE_EUNSUPPORTED;
  const size_t smem = rows_bytes + (sa ? frag_bytes : 0) + (sw ? wtab_bytes : 0);
  hipStream_t s = (hipStream_t)a.stream;
  const int ndt = L.ndt;
#define FE_FL(M)                                                                          \
  if (L.mt == M) {                                                                        \
    if (ndt == 1) {                                                                       \
      if (sa && sw) return launch_fused_one<P, M, 1, true, true>(k, a.ntasks_max, smem, s);             \
      if (sa) return launch_fused_one<P, M, 1, true, false>(k, a.ntasks_max, smem, s);                  \
      if (sw) return launch_fused_one<P, M, 1, false, true>(k, a.ntasks_max, smem, s);                  \
      return launch_fused_one<P, M, 1, false, false>(k, a.ntasks_max, smem, s);                         \
    }                                                                                     \
    if (sa && sw) return launch_fused_one<P, M, 3, true, true>(k, a.ntasks_max, smem, s);               \
    if (sa) return launch_fused_one<P, M, 3, true, false>(k, a.ntasks_max, smem, s);                    \
    if (sw) return launch_fused_one<P, M, 3, false, true>(k, a.ntasks_max, smem, s);                    \
    return launch_fused_one<P, M, 3, false, false>(k, a.ntasks_max, smem, s);                           \
  }
  FE_FL(1) FE_FL(2) FE_FL(3) FE_FL(4) FE_FL(6) FE_FL(8) FE_FL(11)
#undef FE_FL
  return FE_EUNSUPPORTED;
}

}  // namespace fe
