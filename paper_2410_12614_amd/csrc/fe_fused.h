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
#pragma once

#include "fe_cell_kernel.h"

namespace fe {

struct FusedArgs {
  const unsigned char *afrag, *afrag_lo;
  const void *wtab;
  const void *geo;        // FormGeo<T>[n_cells]
  const FusedTask *tasks;
  int ntasks;
  const FusedLane *lanes;
  const uint16_t *srank;  // [pairs][rstride], schedule order: LDS byte offsets of a lane's outputs
  void *values;
  int n_phi, n_q_pad, nks, rstride;
};

// Geometry pass: FP64 geometry of every cell (Section 4.2) and the factors of
// H of one form, with the arithmetic of the cell kernel.
template <class P>
__global__ __launch_bounds__(256) void k_form_geo(const double *coords, int64_t n_cells, int d,
                                                   int nd, const FormHeader *hdr,
                                                   FormGeo<typename P::real> *geo,
                                                   int32_t *status) {
  typedef typename P::real T;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  double G[3][3], adet;
  const bool ok = cell_geometry(d, coords + c * (d + 1) * d, G, adet);
  typename P::hreal Gp[3][3];
  T inv;
  cell_factors<P>(hdr, nd, true, ok, G, adet, 1.0, Gp, inv);
  FormGeo<T> r;
  r.g[0] = Gp[0][0];
  r.g[1] = Gp[0][1];
  r.g[2] = Gp[0][2];
  r.g[3] = Gp[1][1];
  r.g[4] = Gp[1][2];
  r.g[5] = Gp[2][2];
  r.inv = inv;
  r.pad = 0;
  geo[c] = r;
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

template <class P, int MT, int NDT, bool STAGE_A, int NW>
__global__ __launch_bounds__(NW * 64) void fused_kernel(FusedArgs a) {
  typedef typename P::real T;
  typedef typename P::hreal HT;  // weighted table and H formation
  typedef typename P::acc ACC;
  typedef typename P::frag FRAG;
  typedef FormGeo<T> GEO;
  constexpr int KPL = P::KPL;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = lane & 15, kb = lane >> 4;
  const int nphi = a.n_phi, n_q_pad = a.n_q_pad, nks = a.nks;
  const int nqc = n_q_pad / P::KSTEP;

  // Staged weighted table, one row per j holding (chunk qc, slab t, K-slot
  // entries) in the order the K loop reads them, so that a lane's reads are
  // one base plus constant offsets.  Rows are padded by 16 bytes: the 16
  // lanes of a K-slot read 16 different rows j at the same offset, which
  // would fall into the same LDS banks with a power-of-two row stride.
  constexpr int WPAD = 16 / sizeof(HT);
  const int jstride = NDT * n_q_pad + WPAD;
  const size_t frag_bytes = STAGE_A ? (size_t)MT * nks * 64 * sizeof(FRAG) : 0;
  const size_t wtab_bytes = (size_t)nphi * jstride * sizeof(HT);
  unsigned char *s_af = smem;
  unsigned char *s_afl = smem + frag_bytes;
  HT *s_wt = (HT *)(smem + frag_bytes * (P::SPLIT ? 2 : 1));
  T *rowbuf = (T *)(smem + frag_bytes * (P::SPLIT ? 2 : 1) + wtab_bytes) +
              (size_t)wave * (FUSED_SPAN + 64);

  if constexpr (STAGE_A) {
    const size_t n16 = frag_bytes / 16;
    for (size_t t = tid; t < n16; t += NW * 64) ((uint4 *)s_af)[t] = ((const uint4 *)a.afrag)[t];
    if constexpr (P::SPLIT)
      for (size_t t = tid; t < n16; t += NW * 64) ((uint4 *)s_afl)[t] = ((const uint4 *)a.afrag_lo)[t];
  }
  {
    // global table [t][j][n_q_pad], copied by 16-byte pieces (one piece never
    // straddles two K-steps: a K-step is 16, 32 or 128 bytes)
    constexpr int E = 16 / sizeof(HT);
    const int per_row = n_q_pad / E;
    const int nrows = NDT * nphi;
    for (int u = tid; u < nrows * per_row; u += NW * 64) {
      const int row = u / per_row, q = (u - row * per_row) * E;
      const int t = row / nphi, j = row - t * nphi;
      const int qc = q / P::KSTEP, qq = q - qc * P::KSTEP;
      *(uint4 *)(s_wt + (size_t)j * jstride + (qc * NDT + t) * P::KSTEP + qq) =
          ((const uint4 *)a.wtab)[u];
    }
  }
  __syncthreads();

  const GEO *geo = (const GEO *)a.geo;
  const int ntasks = a.ntasks;
  const int stride = gridDim.x * NW;
  int task = blockIdx.x * NW + wave;

  // lane record (two words) and factors of slot `lane` of the wave's task
  FusedTask tk{};
  int lw0 = -1, lw1 = 0;
  GEO gg{};
  if (task < ntasks) {
    tk = a.tasks[task];
    if (lane < tk.nt * 16) {
      const FusedLane l = a.lanes[(size_t)tk.t0 * 16 + lane];
      lw0 = l.cell;
      lw1 = lane_word1(l);
    }
    if (lw0 >= 0) gg = geo[lw0];
  }

  while (task < ntasks) {
    const int nt = tk.nt, span = tk.span, p0 = tk.p0, pre = tk.pre;
    const int64_t base = tk.base;
    const int cw0 = lw0, cw1 = lw1;
    const GEO cg = gg;
    const int next = task + stride;
    const bool has_next = next < ntasks;
    if (has_next) tk = a.tasks[next];

    {
      constexpr int E4 = 16 / sizeof(T);  // elements per 16-byte store
      const int n16 = (span + E4 - 1) / E4;
      for (int t = lane; t < n16; t += 64) ((uint4 *)rowbuf)[t] = uint4{0, 0, 0, 0};
    }

    for (int tl = 0; tl < nt; ++tl) {
      // this lane's column: slot 16 tl + n of the task
      const int src = 16 * tl + n;
      const int cell = __shfl(cw0, src);
      const int w1 = __shfl(cw1, src);
      const int jv = (w1 >> 16) & 0xff, rnd = (w1 >> 24) & 0xf;
      HT Gs[3][3];  // values of the half type when H is formed in half: exact
      {
        const HT g0 = (HT)shfl_t(cg.g[0], src), g1 = (HT)shfl_t(cg.g[1], src);
        const HT g2 = (HT)shfl_t(cg.g[2], src), g3 = (HT)shfl_t(cg.g[3], src);
        const HT g4 = (HT)shfl_t(cg.g[4], src), g5 = (HT)shfl_t(cg.g[5], src);
        Gs[0][0] = g0; Gs[0][1] = g1; Gs[0][2] = g2;
        Gs[1][0] = g1; Gs[1][1] = g3; Gs[1][2] = g4;
        Gs[2][0] = g2; Gs[2][1] = g4; Gs[2][2] = g5;
      }
      const T inv = shfl_t(cg.inv, src);

      // LDS byte offsets of this lane's outputs inside the row buffer, in
      // lane order (four per row tile: one 8-byte load), loaded before the
      // contraction so that their latency hides behind it.  Padding rows
      // point at the lane's private slot; idle lanes never scatter.
      int addr[MT][4];
      {
        const int pair = cell < 0 ? 0 : p0 + ((pre >> (8 * tl)) & 0xff) + n;
        const uint16_t *rk = a.srank + (size_t)pair * a.rstride + 4 * kb;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const uint2 u = *(const uint2 *)(rk + mt * 16);
          addr[mt][0] = (int)(u.x & 0xffff);
          addr[mt][1] = (int)(u.x >> 16);
          addr[mt][2] = (int)(u.y & 0xffff);
          addr[mt][3] = (int)(u.y >> 16);
        }
      }
      // next task's lane records, behind the first tile's contraction
      if (tl == 0 && has_next) {
        lw0 = -1;
        lw1 = 0;
        if (lane < tk.nt * 16) {
          const FusedLane l = a.lanes[(size_t)tk.t0 * 16 + lane];
          lw0 = l.cell;
          lw1 = lane_word1(l);
        }
      }

      ACC acc[MT];
      ACC acc2[P::SPLIT ? MT : 1];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        acc[mt] = ACC{0, 0, 0, 0};
        if constexpr (P::SPLIT) acc2[mt] = ACC{0, 0, 0, 0};
      }
      // K = (s, q) walked q-chunk outer, s inner, as in the cell kernel
      const HT *wcol = s_wt + (size_t)jv * jstride + kb * KPL;
      for (int qc = 0; qc < nqc; ++qc) {
        if constexpr (P::H16) {
          half8_t wv[NDT];
#pragma unroll
          for (int t = 0; t < NDT; ++t) wv[t] = *(const half8_t *)(wcol + (qc * NDT + t) * P::KSTEP);
#pragma unroll
          for (int s = 0; s < NDT; ++s) {
            const half8_t hf = form_h16<NDT>(Gs[s], wv);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              const size_t fi = frag_slot(mt, s, qc, MT, NDT) * 64 + lane;
              FRAG af;
              if constexpr (STAGE_A) af = lds_frag<P>(s_af, fi);
              else af = P::load(a.afrag, fi);
              acc[mt] = P::mma(af, hf, acc[mt]);
            }
          }
        } else {
          T wv[NDT][KPL];
#pragma unroll
          for (int t = 0; t < NDT; ++t) load_w<T, KPL>(wcol + (qc * NDT + t) * P::KSTEP, wv[t]);
#pragma unroll
          for (int s = 0; s < NDT; ++s) {
            T h[KPL];
            form_h<T, NDT, KPL>(Gs[s], wv, h);
            if constexpr (P::SPLIT) {
              FRAG hh, hl;
              P::pack2(h, hh, hl);
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) {
                const size_t fi = frag_slot(mt, s, qc, MT, NDT) * 64 + lane;
                FRAG af, al;
                if constexpr (STAGE_A) {
                  af = lds_frag<P>(s_af, fi);
                  al = lds_frag<P>(s_afl, fi);
                } else {
                  af = P::load(a.afrag, fi);
                  al = P::load(a.afrag_lo, fi);
                }
                acc[mt] = P::mma(af, hh, acc[mt]);
                acc2[mt] = P::mma(af, hl, acc2[mt]);
                acc2[mt] = P::mma(al, hh, acc2[mt]);
              }
            } else {
              const FRAG hf = P::pack(h);
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) {
                const size_t fi = frag_slot(mt, s, qc, MT, NDT) * 64 + lane;
                FRAG af;
                if constexpr (STAGE_A) af = lds_frag<P>(s_af, fi);
                else af = P::load(a.afrag, fi);
                acc[mt] = P::mma(af, hf, acc[mt]);
              }
            }
          }
        }
      }

      // next task's factors: its lane records have arrived by now
      if (tl == 0 && has_next) {
        gg = GEO{};
        if (lw0 >= 0) gg = geo[lw0];
      }

      // scatter into the owned rows, one round per repeated row; within a
      // round every lane adds to a different entry (padding rows update the
      // lane's private slot instead: no branch per entry)
      T val[MT][4];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T v = acc[mt][q];
          if constexpr (P::SPLIT) v += acc2[mt][q] * (T)(1.0 / 2048.0);
          val[mt][q] = v * inv;
        }
      unsigned char *rb = (unsigned char *)rowbuf;
      // the tile's last round, the same in every lane record of the tile
      const int maxr = __builtin_amdgcn_readfirstlane((int)((unsigned)w1 >> 28));
      for (int r = 0; r <= maxr; ++r) {
        if (rnd == r) {
          // read all, then write all: a lane's entries are distinct and the
          // lanes of one round hold distinct rows
          T old[MT][4];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) old[mt][q] = *(const T *)(rb + addr[mt][q]);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) *(T *)(rb + addr[mt][q]) = old[mt][q] + val[mt][q];
        }
      }
    }
    T *V = (T *)a.values + base;
    for (int t = lane; t < span; t += 64) V[t] = rowbuf[t];
    task = next;
  }
}

template <class P, int MT, int NDT, bool SA, int NW>
static fe_status launch_fused_one(const FusedArgs &k, size_t smem, hipStream_t s) {
  auto kern = fused_kernel<P, MT, NDT, SA, NW>;
  if (smem > 65536 && hipFuncSetAttribute((const void *)kern,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)smem) != hipSuccess)
    return FE_EHIP;
  int dev = 0, ncu = 256, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, NW * 64, smem) !=
          hipSuccess)
    return FE_EHIP;
  if (per_cu < 1) return FE_EUNSUPPORTED;
  const int64_t need = ((int64_t)k.ntasks + NW - 1) / NW;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)ncu * per_cu));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), smem, s, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

template <class P, int MT, int NDT>
static fe_status launch_fused_nw(const FusedArgs &k, const FormLayout &L, hipStream_t s) {
  // the most waves per workgroup that fit, B^T fragments staged when they fit
  if (fused_lds(L, 16, true) <= FUSED_LDS_BUDGET)
    return launch_fused_one<P, MT, NDT, true, 16>(k, fused_lds(L, 16, true), s);
  if (fused_lds(L, 12, true) <= FUSED_LDS_BUDGET)
    return launch_fused_one<P, MT, NDT, true, 12>(k, fused_lds(L, 12, true), s);
  if (fused_lds(L, 8, true) <= FUSED_LDS_BUDGET)
    return launch_fused_one<P, MT, NDT, true, 8>(k, fused_lds(L, 8, true), s);
  if (fused_lds(L, 8, false) <= FUSED_LDS_BUDGET)
    return launch_fused_one<P, MT, NDT, false, 8>(k, fused_lds(L, 8, false), s);
  if (fused_lds(L, 4, false) <= FUSED_LDS_BUDGET)
    return launch_fused_one<P, MT, NDT, false, 4>(k, fused_lds(L, 4, false), s);
  return FE_EUNSUPPORTED;
}

template <class P>
fe_status launch_fused_impl(const FusedLaunch &a) {
  typedef typename P::real T;
  const FormLayout &L = *a.L;
  hipStream_t s = (hipStream_t)a.stream;
  if (!fused_eligible(L)) return FE_EUNSUPPORTED;
  if (a.n_cells > 0) {
    hipLaunchKernelGGL(k_form_geo<P>, dim3((unsigned)((a.n_cells + 255) / 256)), dim3(256), 0, s,
                       a.coords, a.n_cells, L.d, L.nd, (const FormHeader *)a.form_buf,
                       (FormGeo<T> *)a.geo, a.status);
    if (hipGetLastError() != hipSuccess) return FE_EHIP;
  }
  if (a.ntasks <= 0) return FE_OK;
  FusedArgs k;
  k.afrag = a.form_buf + L.off_afrag;
  k.afrag_lo = a.form_buf + L.off_afrag_lo;
  k.wtab = a.form_buf + L.off_wtab;
  k.geo = a.geo;
  k.tasks = a.tasks;
  k.ntasks = (int)a.ntasks;
  k.lanes = a.lanes;
  k.srank = a.srank;
  k.values = a.values;
  k.n_phi = L.n_phi;
  k.n_q_pad = L.n_q_pad;
  k.nks = L.nks;
  k.rstride = a.rstride;
#define FE_FL(M)                                               \
  if (L.mt == M) {                                             \
    if (L.ndt == 1) return launch_fused_nw<P, M, 1>(k, L, s);  \
    return launch_fused_nw<P, M, 3>(k, L, s);                  \
  }
  FE_FL(1) FE_FL(2) FE_FL(3) FE_FL(4) FE_FL(6) FE_FL(8) FE_FL(11)
#undef FE_FL
  return FE_EUNSUPPORTED;
}

}  // namespace fe
