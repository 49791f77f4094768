// Whole-cell kernel: one wave computes the complete local matrix of one cell
// at a time, A_K = sum_s B_s^T H_s with H_s = sum_t C_st B_t (Algorithm 1,
// the one-H-per-s reading of the remark after it), in FP16 storage with
// FP32 accumulation on the matrix cores.
//
// The B^T fragments of a quadrature chunk (32 points, every derivative slab
// s and row tile) are the left operand of the contraction AND, lane for
// lane, the table H is formed from: in the 16 x 16 x 32 instruction the
// left operand of row tile I and the right operand of column tile J have the
// same lane layout (lane l: row / column l % 16, K entries 8 (l / 16) + e),
// so lane l forms its entries of H_s(:, J) from its own registers of the
// fragments of tile J,
//
//     H_s(q, j) = sum_t c_st(q) F_t(q, j),   c_st(q) = w_q z(X_q) G_st,
//
// with no data exchanged between lanes.  The chunk's fragments are read once
// from a three-slot LDS ring that the workgroup fills from the (L2-resident)
// form buffer; every wave of the workgroup walks the same chunks.  The
// forms are symmetric, so only the tiles (I, J) with I <= J are contracted
// and the tile (I, J) is also stored transposed: MT (MT + 1) / 2 tiles
// instead of MT^2.
//
// Scaling: F = 2^b B (the form buffer's exact power of two, |F| < 2^15);
// c_st = fl16(2^-e1 w_q z_q) fl16(2^e2 G_st) with 2^-e1 max_q |w_q z_q| < 1
// and 2^e2 max_s sum_t |G_st| < 1, so |H| < 2^15 in half arithmetic; the FP32
// result is multiplied by the exact 2^(e1 - e2 - 2b).  Geometry is FP64 (or
// the form's geometry mode) per cell; the coefficient at the points comes
// from k_coeff_points (single precision, u_p = u^2 relative to FP16).
#pragma once

#include "fe_cell_kernel.h"

namespace fe {

// ---- coefficient at the quadrature points (FE function evaluation) ----
// z_K(X_q) = sum_k z_{dof(K,k)} phi_k(X_q) for every cell, as a batched
// product (n_q x n_phi) (n_phi x cells) on the FP32 matrix cores
// (16 x 16 x 4): each wave takes 16 NG cells along N, the value table
// phi_k(X_q) is the left operand (rows q).  Writes z [n_cells][n_q_pad]
// (zero past n_q) and max_q |z_K(X_q)| per cell.
template <int KS, int NG>
__global__ __launch_bounds__(256) void k_coeff_points(const float *vtab, const int32_t *dofmap,
                                                      const double *coeff, int64_t n_cells,
                                                      int64_t n_dofs, int n_phi, int n_q, int n_q_pad,
                                                      float *zpt, float *zmax, int32_t *status) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 15, kb = lane >> 4;
  const int64_t cell0 = ((int64_t)blockIdx.x * 4 + wave) * 16 * NG;
  if (cell0 >= n_cells) return;
  // right operands: this lane's cell (column c) at the K entries 4 ks + kb
  float zk[NG][KS];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int64_t cell = cell0 + 16 * g + c;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + kb;
      float v = 0.0f;
      if (cell < n_cells && k < n_phi) {
        const int32_t gd = dofmap[cell * n_phi + k];
        if (gd >= 0 && gd < n_dofs) v = (float)coeff[gd];
        else atomicOr(status, STATUS_BAD_DOF);
      }
      zk[g][ks] = v;
    }
  }
  float zm[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) zm[g] = 0.0f;
  // left operands of q tile qt (row 16 qt + c, K entries 4 ks + kb), the
  // next tile's loaded while the current one is contracted
  auto load_a = [&](int qt, float (&av)[KS]) {
    const int q = 16 * qt + c;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + kb;
      av[ks] = (q < n_q && k < n_phi) ? vtab[(size_t)q * n_phi + k] : 0.0f;
    }
  };
  const int nqt = n_q_pad / 16;
  float av[KS];
  load_a(0, av);
  for (int qt = 0; qt < nqt; ++qt) {
    float an[KS];
    if (qt + 1 < nqt) load_a(qt + 1, an);
    f32x4_t acc[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[g] = f32x4_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int g = 0; g < NG; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks], zk[g][ks], acc[g], 0, 0, 0);
    }
    // lane: column c (the cell), rows 16 qt + 4 kb + r
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int64_t cell = cell0 + 16 * g + c;
      if (cell < n_cells)
        *(float4 *)(zpt + cell * n_q_pad + 16 * qt + 4 * kb) =
            float4{acc[g][0], acc[g][1], acc[g][2], acc[g][3]};
#pragma unroll
      for (int r = 0; r < 4; ++r) zm[g] = fmaxf(zm[g], fabsf(acc[g][r]));
    }
    if (qt + 1 < nqt)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[ks] = an[ks];
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    float m = zm[g];
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    const int64_t cell = cell0 + 16 * g + c;
    if (kb == 0 && cell < n_cells) zmax[cell] = m;
  }
}

struct CwArgs {
  const unsigned char *afrag;  // B^T fragments [qc][s][mt][lane] (half8), chunk-major
  const double *wq;            // quadrature weights [n_q_pad]
  const FormHeader *hdr;
  int32_t *status;
  const double *coords;
  const float *zpt;   // [n_cells][n_q_pad] coefficient at the points, or null (z = 1)
  const float *zmax;  // [n_cells] max_q |z|, or null
  float *A;           // [n_cells][n_phi][n_phi]
  int64_t n_cells;
  int d, n_phi, n_q, n_q_pad;
};

// Index of the symmetric tile pair (I, J), I <= J, in row-major order of
// the upper triangle of an MT x MT tile grid.
template <int MT>
__device__ __forceinline__ constexpr int pair_index(int I, int J) {
  return I * MT - I * (I - 1) / 2 + (J - I);
}

// Per-cell factors of one wave's current cell: the scaled geometry tensor
// in half (both halves of a register), the scale of w z and the exact
// inverse of all scales.
template <int NDT>
struct CwCell {
  half2_t g2[NDT == 1 ? 1 : 6];
  float zsc, inv;
  bool ok;
};

template <int NDT, bool COEFF>
__device__ __forceinline__ CwCell<NDT> cw_cell(const CwArgs &a, int64_t ce) {
  CwCell<NDT> r;
  double G[3][3], adet;
  r.ok = cell_geometry_mode(a.hdr->geom, a.d, a.coords + ce * (a.d + 1) * a.d, G, adet);
  double gabs = adet;
  if constexpr (NDT == 3) {
    gabs = 0.0;
    for (int s = 0; s < 3; ++s) gabs = fmax(gabs, fabs(G[s][0]) + fabs(G[s][1]) + fabs(G[s][2]));
  }
  const double zm = COEFF ? (double)a.zmax[ce] : 1.0;
  const double wzmax = a.hdr->max_w * zm;
  const int e1 = (wzmax > 0.0 && isfinite(wzmax)) ? 1 + ilogb(wzmax) : 0;
  const int e2 = (gabs > 0.0 && isfinite(gabs)) ? -1 - ilogb(gabs) : 0;
#pragma unroll
  for (int s = 0; s < NDT; ++s)
#pragma unroll
    for (int t = s; t < NDT; ++t) {
      double v = NDT == 1 ? adet : G[s][t];
      v = r.ok ? ldexp(v, e2) : NAN;
      r.g2[NDT == 1 ? 0 : sym_comp(s, t)] = half2_t{(_Float16)v, (_Float16)v};
    }
  const double bsc = a.hdr->b_scale;
  r.zsc = (float)ldexp(1.0, -e1);
  r.inv = (float)(ldexp(1.0, e1 - e2) / (bsc * bsc));
  return r;
}

// Chunks flow through a three-slot LDS ring by direct global-to-LDS loads
// (no registers): while chunk g is contracted, chunk g + 2 travels into the
// slot chunk g - 1 left; the chunk's fragments are read from LDS at its
// start, its coefficient values from memory.  One
// barrier per chunk; every wave of a workgroup runs the same number of
// chunks (the last round's waves without a cell compute a clamped cell and
// store nothing), so the barriers match.
// s_waitcnt immediate (gfx9 encoding) waiting until at most n vector
// memory operations of this wave are outstanding (LDS and export counters
// left free)
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14); }

template <int MT, int NDT, bool COEFF, int NW>
__global__ __launch_bounds__(NW * 64) void cellwise_kernel(CwArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NT = NW * 64;
  constexpr int NP = MT * (MT + 1) / 2;
  constexpr int CH16 = NDT * MT * 64;         // 16-byte pieces of one chunk (a multiple of 64)
  constexpr int PRE = (CH16 + NT - 1) / NT;  // pieces per thread
  constexpr int PRE_MIN = CH16 / NT;         // direct loads every wave issues per chunk
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c = lane & 15, kb = lane >> 4;
  const int nphi = a.n_phi, n_q_pad = a.n_q_pad;
  const int nqc = n_q_pad / 32;
  uint4 *ring = (uint4 *)smem;                  // [3][CH16]
  float *wl = (float *)(smem + 3 * CH16 * 16);  // [n_q_pad]
  const uint4 *src = (const uint4 *)a.afrag;

  const int64_t per_round = (int64_t)gridDim.x * NW;
  const int rounds = (int)((a.n_cells + per_round - 1) / per_round);
  const int total = rounds * nqc;  // chunks this wave walks
  // table chunk tc into ring slot sl: each wave moves whole runs of 64
  // pieces, lane l the piece base + l
  auto fill = [&](int tc, int sl) {
    const uint4 *from = src + (size_t)tc * CH16;
    uint4 *to = ring + sl * CH16;
#pragma unroll
    for (int p = 0; p < PRE; ++p) {
      const int e0 = p * NT + wave * 64;  // wave-uniform
      if (e0 < CH16)
        __builtin_amdgcn_global_load_lds(
            (const void __attribute__((address_space(1))) *)(from + e0 + lane),
            (void __attribute__((address_space(3))) *)(to + e0), 16, 0, 0);
    }
  };

  for (int i = tid; i < n_q_pad; i += NT) wl[i] = (float)a.wq[i];
  fill(0, 0);
  if (total > 1) fill(1 % nqc, 1);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // walk position g: its ring slot g % 3, and the table chunk and slot of
  // g + 2 (counters, no divisions in the loop)
  int g = 0, slot = 0, fslot = 2, fchunk = 2 % nqc;
  for (int rd = 0; rd < rounds; ++rd) {
    const int64_t cell = (int64_t)rd * per_round + (int64_t)blockIdx.x * NW + wave;
    const bool valid = cell < a.n_cells;
    const int64_t ce = valid ? cell : a.n_cells - 1;
    const CwCell<NDT> cf = cw_cell<NDT, COEFF>(a, ce);
    const float *zrow = COEFF ? a.zpt + ce * n_q_pad + 8 * kb : nullptr;
    f32x4_t acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = f32x4_t{0, 0, 0, 0};

    for (int qc = 0; qc < nqc; ++qc, ++g) {
      // the chunk's coefficient values (issued before the direct loads:
      // vector memory operations complete in order, so using these does not
      // wait for the ring)
      float4 z0 = {1, 1, 1, 1}, z1 = {1, 1, 1, 1};
      if constexpr (COEFF) {
        z0 = *(const float4 *)(zrow + qc * 32);
        z1 = *(const float4 *)(zrow + qc * 32 + 4);
      }
      // slot (g + 2) % 3 last held chunk g - 1, which every wave finished
      // before the barrier that closed it
      if (g + 2 < total) fill(fchunk, fslot);
      fchunk = fchunk + 1 == nqc ? 0 : fchunk + 1;
      fslot = fslot == 2 ? 0 : fslot + 1;
      // the chunk's fragments
      half8_t F[NDT][MT];
      const uint4 *cur = ring + slot * CH16;
      slot = slot == 2 ? 0 : slot + 1;
#pragma unroll
      for (int s = 0; s < NDT; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const uint4 u = cur[(s * MT + mt) * 64 + lane];
          F[s][mt] = *reinterpret_cast<const half8_t *>(&u);
        }
      // this lane's eight points: w z scaled, rounded in pairs
      const float *w8 = wl + qc * 32 + 8 * kb;
      const float zc[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
      half2_t wz[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        wz[p] = half2_t{(_Float16)(w8[2 * p] * zc[2 * p] * cf.zsc),
                        (_Float16)(w8[2 * p + 1] * zc[2 * p + 1] * cf.zsc)};
#pragma unroll
      for (int s = 0; s < NDT; ++s) {
        half2_t cst[NDT][4];
#pragma unroll
        for (int t = 0; t < NDT; ++t)
#pragma unroll
          for (int p = 0; p < 4; ++p) cst[t][p] = wz[p] * cf.g2[NDT == 1 ? 0 : sym_comp(s, t)];
#pragma unroll
        for (int J = 0; J < MT; ++J) {
          half8_t h;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            half2_t x = half2_t{F[0][J][2 * p], F[0][J][2 * p + 1]} * cst[0][p];
#pragma unroll
            for (int t = 1; t < NDT; ++t)
              x = __builtin_elementwise_fma(half2_t{F[t][J][2 * p], F[t][J][2 * p + 1]}, cst[t][p], x);
            h[2 * p] = x[0];
            h[2 * p + 1] = x[1];
          }
#pragma unroll
          for (int I = 0; I <= J; ++I)
            acc[pair_index<MT>(I, J)] =
                __builtin_amdgcn_mfma_f32_16x16x32_f16(F[s][I], h, acc[pair_index<MT>(I, J)], 0, 0, 0);
        }
      }
      // chunk g + 1 (loaded during chunk g - 1) has landed: every vector
      // memory operation but this chunk's last PRE_MIN direct loads is done
      // (chunk g + 2's loads may stay in flight through chunk g + 1); then
      // every wave's, at the barrier
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(PRE_MIN));
      __syncthreads();
    }

    // ---- the tiles (I, J), I <= J (lane: A(i, j) for j = 16 J + c,
    // i = 16 I + 4 kb + r), stored as rows j (four consecutive i: one
    // 16-byte store) and, off the diagonal, as rows i ----
    if (valid) {
      if (!cf.ok && lane == 0) atomicOr(a.status, STATUS_DEGENERATE);
      float *A = a.A + ce * (int64_t)nphi * nphi;
#pragma unroll
      for (int I = 0; I < MT; ++I)
#pragma unroll
        for (int J = I; J < MT; ++J) {
          const f32x4_t v = acc[pair_index<MT>(I, J)] * cf.inv;
          const int j = 16 * J + c, i0 = 16 * I + 4 * kb;
          if (j < nphi) {
            float *row = A + (size_t)j * nphi;
            if (i0 + 3 < nphi) {
              *(f4u_t *)(row + i0) = f4u_t{v[0], v[1], v[2], v[3]};
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (i0 + r < nphi) row[i0 + r] = v[r];
            }
            if (I != J) {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (i0 + r < nphi) A[(size_t)(i0 + r) * nphi + j] = v[r];
            }
          }
        }
    }
  }
}

template <int MT, int NDT, bool COEFF, int NW>
static fe_status launch_cellwise_one(const CellwiseLaunch &c, const CwArgs &k) {
  auto kern = cellwise_kernel<MT, NDT, COEFF, NW>;
  const size_t smem = (size_t)3 * NDT * MT * 64 * 16 + (size_t)c.L->n_q_pad * sizeof(float);
  LaunchInfo li;
  if (launch_info((const void *)kern, NW * 64, smem, &li) != FE_OK) return FE_EHIP;
  if (li.per_cu < 1) return FE_EUNSUPPORTED;
  const int64_t need = (c.n_cells + NW - 1) / NW;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)li.ncu * li.per_cu));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), smem, (hipStream_t)c.stream, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

template <int KS>
static fe_status launch_coeff_points(const CellwiseLaunch &c) {
  const FormLayout &L = *c.L;
  constexpr int NG = 2;
  const int64_t waves = (c.n_cells + 16 * NG - 1) / (16 * NG);
  hipLaunchKernelGGL((k_coeff_points<KS, NG>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0,
                     (hipStream_t)c.stream, (const float *)(c.form_buf + L.off_vtab), c.dofmap, c.coeff, c.n_cells,
                     c.n_dofs, L.n_phi, L.n_q, L.n_q_pad, c.zpt, c.zmax, c.status);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

inline fe_status launch_cellwise(const CellwiseLaunch &c) {
  const FormLayout &L = *c.L;
  if (!cellwise_eligible(L)) return FE_EUNSUPPORTED;
  if (c.n_cells == 0) return FE_OK;
  const bool coeff = c.coeff != nullptr;
  if (coeff) {
    if (!c.zpt || !c.zmax) return FE_EINVAL;
    const int ks = (L.n_phi + 3) / 4;
    fe_status st = FE_EUNSUPPORTED;
    if (ks == 21) st = launch_coeff_points<21>(c);
    if (st != FE_OK) return st;
  }
  CwArgs k;
  k.afrag = c.form_buf + L.off_afrag;
  k.wq = (const double *)(c.form_buf + L.off_wq);
  k.hdr = (const FormHeader *)c.form_buf;
  k.status = c.status;
  k.coords = c.coords;
  k.zpt = c.zpt;
  k.zmax = c.zmax;
  k.A = c.A_local;
  k.n_cells = c.n_cells;
  k.d = L.d;
  k.n_phi = L.n_phi;
  k.n_q = L.n_q;
  k.n_q_pad = L.n_q_pad;
  if (L.ndt == 3) {
    if (L.mt == 6)
      return coeff ? launch_cellwise_one<6, 3, true, 8>(c, k) : launch_cellwise_one<6, 3, false, 8>(c, k);
    return FE_EUNSUPPORTED;
  }
  if (coeff) return FE_EUNSUPPORTED;
  switch (L.mt) {
    case 4: return launch_cellwise_one<4, 1, false, 4>(c, k);
    case 6: return launch_cellwise_one<6, 1, false, 4>(c, k);
    case 8: return launch_cellwise_one<8, 1, false, 4>(c, k);
  }
  return FE_EUNSUPPORTED;
}

}  // namespace fe
