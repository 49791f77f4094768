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

// Per-cell factors of the whole-cell kernel: the scaled geometry tensor in
// half (both halves of a register), the scale of w z and the exact inverse
// of all scales.
template <int NDT>
struct CwCell {
  half2_t g2[NDT == 1 ? 1 : 6];
  float zsc, inv;
  bool ok;
};

template <int NDT>
__device__ __forceinline__ CwCell<NDT> cell_scales(const FormHeader *hdr, int d, const double *xc,
                                                   double zm) {
  CwCell<NDT> r;
  double G[3][3], adet;
  r.ok = cell_geometry_mode(hdr->geom, d, xc, G, adet);
  double gabs = adet;
  if constexpr (NDT == 3) {
    gabs = 0.0;
    for (int s = 0; s < 3; ++s) gabs = fmax(gabs, fabs(G[s][0]) + fabs(G[s][1]) + fabs(G[s][2]));
  }
  const double wzmax = hdr->max_w * zm;
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
  const double bsc = hdr->b_scale;
  r.zsc = (float)ldexp(1.0, -e1);
  r.inv = (float)(ldexp(1.0, e1 - e2) / (bsc * bsc));
  return r;
}

// The factors of a coefficient form's cell as the coefficient pass stores
// them (two 16-byte words)
struct CwRec {
  half2_t g2[6];
  float zsc, inv;
};

// ---- coefficient at the quadrature points (FE function evaluation) ----
// z_K(X_q) = sum_k z_{dof(K,k)} phi_k(X_q) for every cell, as a batched
// product (n_q x n_phi) (n_phi x cells) on the FP32 matrix cores
// (16 x 16 x 4): each wave takes 16 NG cells along N, the value table
// phi_k(X_q) is the left operand (rows q).  The four waves of a workgroup
// walk the same 16-point tiles of the table, which they stage in LDS
// together (coalesced loads into registers, written after the current
// tile's products; two LDS buffers, one barrier per tile).  Writes z
// [n_cells][n_q_pad] (zero past n_q) and max_q |z_K(X_q)| per cell, and
// then, one lane per cell, the cell's factors for the whole-cell kernel
// (FP64 geometry, the scales of H; a degenerate cell raises the status
// flag).
template <int KS, int NG>
__global__ __launch_bounds__(256) void k_coeff_points(const float *vtab, const int32_t *dofmap,
                                                      const double *coeff, int64_t n_cells,
                                                      int64_t n_dofs, int n_phi, int n_q, int n_q_pad,
                                                      const FormHeader *hdr, const double *coords,
                                                      int d, float *zpt, float *zmax, CwRec *rec,
                                                      int32_t *status) {
  constexpr int TW = 4 * KS;                 // table row width in LDS (n_phi padded)
  constexpr int TP = (16 * TW + 255) / 256;  // staged values per thread and tile
  __shared__ float vt[2][16 * TW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 15, kb = lane >> 4;
  const int64_t cell0 = ((int64_t)blockIdx.x * 4 + wave) * 16 * NG;
  // (a wave past the cells still stages its share and meets the barriers)
  const bool active = cell0 < n_cells;
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
  // table tile qt (rows 16 qt .. + 15, entries [row][k], zero past n_q and
  // n_phi): this thread's values, then into LDS buffer b
  auto load_t = [&](int qt, float (&pv)[TP]) {
#pragma unroll
    for (int p = 0; p < TP; ++p) {
      const int e = p * 256 + (int)threadIdx.x;
      const int r = e / TW, k = e - r * TW;
      const int q = 16 * qt + r;
      pv[p] = (e < 16 * TW && q < n_q && k < n_phi) ? vtab[(size_t)q * n_phi + k] : 0.0f;
    }
  };
  auto put_t = [&](int b, const float (&pv)[TP]) {
#pragma unroll
    for (int p = 0; p < TP; ++p) {
      const int e = p * 256 + (int)threadIdx.x;
      if (e < 16 * TW) vt[b][e] = pv[p];
    }
  };
  const int nqt = n_q_pad / 16;
  {
    float pv[TP];
    load_t(0, pv);
    put_t(0, pv);
  }
  __syncthreads();
  for (int qt = 0; qt < nqt; ++qt) {
    float pn[TP];
    if (qt + 1 < nqt) load_t(qt + 1, pn);
    // left operands of tile qt: row 16 qt + c, K entries 4 ks + kb
    float av[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) av[ks] = vt[qt & 1][c * TW + 4 * ks + kb];
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
    // the next tile into the other buffer (last read in tile qt - 1, which
    // every wave finished before the barrier that closed it)
    if (qt + 1 < nqt) put_t((qt + 1) & 1, pn);
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    float m = zm[g];
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    const int64_t cell = cell0 + 16 * g + c;
    if (kb == 0 && cell < n_cells) {
      zmax[cell] = m;
      const CwCell<3> r = cell_scales<3>(hdr, d, coords + cell * (d + 1) * d, (double)m);
      CwRec w;
#pragma unroll
      for (int e = 0; e < 6; ++e) w.g2[e] = r.g2[e];
      w.zsc = r.zsc;
      w.inv = r.inv;
      rec[cell] = w;
      if (!r.ok) atomicOr(status, STATUS_DEGENERATE);
    }
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
  const CwRec *rec;   // [n_cells] factors from the coefficient pass, or null (computed here)
  float *A;           // [n_cells][n_phi][n_phi]
  int64_t n_cells;
  int d, n_phi, n_q, n_q_pad;
};

template <int NDT, bool COEFF>
__device__ __forceinline__ CwCell<NDT> cw_cell(const CwArgs &a, int64_t ce) {
  return cell_scales<NDT>(a.hdr, a.d, a.coords + ce * (a.d + 1) * a.d, COEFF ? (double)a.zmax[ce] : 1.0);
}

// Chunks flow through a three-slot LDS ring by direct global-to-LDS loads
// (no registers): while chunk g is contracted, chunk g + 2 travels into the
// slot chunk g - 1 left; the chunk's fragments are read from LDS at its
// start.  One barrier per chunk; every wave of a workgroup runs the same
// number of chunks (the last round's waves without a cell compute a clamped
// cell and store nothing), so the barriers match.
//
// Waits.  The three slots are separate LDS arrays and every read and direct
// load names its slot statically (a cell's chunk loop exists in three
// copies, one per slot of its first chunk, each unrolled by three), so the
// compiler knows that loads into one slot do not alias reads of another and
// does not wait for the prefetch before reading the ring.  Every wave
// issues the same number of direct loads per chunk (PRE: a wave with fewer
// pieces repeats its previous one, and the last two chunks of the walk load
// a spare copy of chunk 0 into the free slot), so the counts of vector
// memory operations are the same on every path.  A coefficient form's cell
// factors (computed by the coefficient pass) and the coefficient values at
// all the cell's points (by direct loads into an LDS row of the wave) are
// loaded while the previous cell's rows are stored.  The explicit wait
// closing a chunk (at most the PRE direct loads just issued outstanding)
// covers the loads of the next chunk, and the barrier after it is a bare
// s_barrier (the workgroup-scope fence of __syncthreads() would wait for
// the prefetch as well).
//
// Stores.  The rows of the local matrix leave in blocks of 16 (rows
// 16 J .. 16 J + 15, contiguous in memory): the tiles (I, J), I <= J, give
// their columns 16 I .. + 15 directly (lane: rows 16 J + c, four
// consecutive columns), the tiles (J, I), I > J, transposed (lane: rows
// 16 J + 4 kb + r, column 16 I + c); both are written into a row block in
// the wave's LDS, which then goes out in 16-byte pieces, consecutive lanes
// on consecutive addresses.  With fewer than 11 row tiles n_phi is a
// multiple of four, so a 16-byte piece is either inside the matrix or not;
// with 11 (P8, n_phi = 165) the block is staged as far into the LDS buffer
// as it starts past a 16-byte boundary in memory, and leaves as a few
// dwords, whole 16-byte pieces and a few dwords.  The 66 accumulator tiles
// of that form take all 256 AGPRs and a few VGPRs; they are read out of
// the AGPRs where they are stored (otherwise the compiler copies them all
// to VGPRs at the end of the chunk loop and spills).
//
// Phases.  Workgroups start their walks a quarter, a half or three
// quarters of a cell apart (a prefix of chunks computed and dropped), so
// that not every wave of the chip stores its rows at the same time: a
// wave's next table load waits for its stores (loads and stores share one
// in-order counter).
// s_waitcnt immediate (gfx9 encoding) waiting until at most n vector
// memory operations of this wave are outstanding (LDS and export counters
// left free)
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14); }

// Workgroup barrier without a memory fence (signal fences emit no
// instruction; they keep the compiler from moving memory operations across)
__device__ __forceinline__ void bare_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int S>
using slot_t = std::integral_constant<int, S>;

// An accumulator tile read out of its AGPRs where it is used (volatile asm,
// AGPR operands), times a scale. Plain code would copy every accumulator
// to VGPRs at the end of the chunk loop, which the forms with 66 tiles do
// not have room for. (The MFMA result hazard is the caller's: the
// compiler does not pad inline asm.)
__device__ __forceinline__ f32x4_t agpr_tile_scaled(const f32x4_t &x, float s) {
  float y0, y1, y2, y3;
  asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(y0) : "a"(x[0]));
  asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(y1) : "a"(x[1]));
  asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(y2) : "a"(x[2]));
  asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(y3) : "a"(x[3]));
  return f32x4_t{y0 * s, y1 * s, y2 * s, y3 * s};
}

constexpr int CW_ZMAX = 512;  // points of a coefficient form (n_q_pad) the LDS row holds

// Accumulator of the symmetric tile (I, J), I <= J, column by column.
__device__ __forceinline__ constexpr int tile_index(int I, int J) { return J * (J + 1) / 2 + I; }

template <int MT, int NDT, bool COEFF, int NW>
__global__ __launch_bounds__(NW * 64) void cellwise_kernel(CwArgs a) {
  constexpr int NT = NW * 64;
  constexpr int NP = MT * (MT + 1) / 2;
  constexpr int CH16 = NDT * MT * 64;        // 16-byte pieces of one chunk (a multiple of 64)
  constexpr int PRE = (CH16 + NT - 1) / NT;  // direct loads per wave and chunk
  static_assert(CH16 >= NT, "a chunk covers every thread at least once");
  __shared__ uint4 ring0[CH16], ring1[CH16], ring2[CH16];
  // a wave's row block (16 rows x n_phi)
  __shared__ float4 rbuf[NW][16 * MT * 4];
  __shared__ float zbuf[COEFF ? NW : 1][COEFF ? CW_ZMAX : 4];
  extern __shared__ float wl[];  // quadrature weights [n_q_pad]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c = lane & 15, kb = lane >> 4;
  const int nphi = a.n_phi, n_q_pad = a.n_q_pad;
  const int nqc = n_q_pad / 32;
  const uint4 *src = (const uint4 *)a.afrag;
  float *rb = (float *)rbuf[wave];

  const int64_t per_round = (int64_t)gridDim.x * NW;
  const int rounds = (int)((a.n_cells + per_round - 1) / per_round);
  // workgroups start their walks at four phases of a cell: a prefix of
  // the last `off` chunks of a cell, computed and dropped, so that the
  // stores at the ends of cells do not come from every workgroup at once
  // (a wave's next table load waits for its stores: one in-order counter)
  const int off = (((int)blockIdx.x >> 3) & 3) * nqc / 4;
  const int total = off + rounds * nqc;  // chunks this wave walks
  auto cell_of = [&](int rd) -> int64_t {
    const int64_t cell = (int64_t)rd * per_round + (int64_t)blockIdx.x * NW + wave;
    return cell < a.n_cells ? cell : a.n_cells - 1;
  };
  // table chunk tc into ring slot S: each wave moves whole runs of 64
  // pieces, lane l the piece base + l; a run past the chunk repeats the
  // wave's previous run (same data to the same place)
  auto fill = [&](int tc, auto sl) {
    constexpr int S = decltype(sl)::value;
    uint4 *to = S == 0 ? ring0 : S == 1 ? ring1 : ring2;
    const uint4 *from = src + (size_t)tc * CH16;
#pragma unroll
    for (int p = 0; p < PRE; ++p) {
      int e0 = p * NT + wave * 64;  // wave-uniform
      if (e0 >= CH16) e0 -= NT;
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1))) *)(from + e0 + lane),
          (void __attribute__((address_space(3))) *)(to + e0), 16, 0, 0);
    }
  };
  // coefficient values at all points of cell ce into the wave's LDS row:
  // CW_ZMAX / 256 direct loads, lanes past the row repeat its last piece
  // into the unused end of the LDS row
  auto load_z = [&](int64_t ce) {
    const uint4 *zr = (const uint4 *)(a.zpt + ce * n_q_pad);
    const int last = n_q_pad / 4 - 1;
#pragma unroll
    for (int p = 0; p < CW_ZMAX / 256; ++p)
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1))) *)(zr + min(64 * p + lane, last)),
          (void __attribute__((address_space(3))) *)((uint4 *)zbuf[wave] + 64 * p), 16, 0, 0);
  };
  auto load_rec = [&](int64_t ce, uint4 &r0, uint4 &r1) {
    const uint4 *rp = (const uint4 *)(a.rec + ce);
    r0 = rp[0];
    r1 = rp[1];
  };

  for (int i = tid; i < n_q_pad; i += NT) wl[i] = (float)a.wq[i];
  // walk position g holds chunk (g - off) mod nqc
  fill((nqc - off) % nqc, slot_t<0>());
  fill((nqc - off + 1) % nqc, slot_t<1>());
  // prefetched: the next cell's factors (and its coefficient values)
  uint4 rn0 = {0, 0, 0, 0}, rn1 = {0, 0, 0, 0};
  if constexpr (COEFF) {
    load_z(cell_of(0));
    load_rec(cell_of(0), rn0, rn1);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // (round -1: the prefix, as a cell past the end)
  for (int rd = off > 0 ? -1 : 0; rd < rounds; ++rd) {
    const int64_t cell = rd < 0 ? a.n_cells : (int64_t)rd * per_round + (int64_t)blockIdx.x * NW + wave;
    const bool valid = cell < a.n_cells;
    const int64_t ce = valid ? cell : a.n_cells - 1;
    const int64_t ce_next = cell_of(rd + 1 < rounds ? rd + 1 : rd);
    CwCell<NDT> cf;
    if constexpr (COEFF) {
      CwRec r;
      *reinterpret_cast<uint4 *>(&r) = rn0;
      *(reinterpret_cast<uint4 *>(&r) + 1) = rn1;
#pragma unroll
      for (int e = 0; e < (NDT == 1 ? 1 : 6); ++e) cf.g2[e] = r.g2[e];
      cf.zsc = r.zsc;
      cf.inv = r.inv;
      cf.ok = true;  // the coefficient pass raised the flag
    } else {
      cf = cw_cell<NDT, COEFF>(a, ce);
    }
    f32x4_t acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = f32x4_t{0, 0, 0, 0};
    const int g0 = off + rd * nqc;      // walk position of the cell's chunk 0
    const int q0 = rd < 0 ? nqc - off : 0;  // its first chunk walked

    // chunk qc of the cell (walk position g0 + qc) from slot S; chunk
    // g0 + qc + 2 into slot (S + 2) % 3
    auto step = [&](int qc, auto sl) {
      constexpr int S = decltype(sl)::value;
      const uint4 *cur = S == 0 ? ring0 : S == 1 ? ring1 : ring2;
      // the direct loads of chunk g + 2 into the slot chunk g - 1 left
      // (every wave finished that before the barrier that closed it; past
      // the walk's end a spare copy of chunk 0)
      {
        const int g = g0 + qc;
        int fc = qc + 2;
        if (fc >= nqc) fc -= nqc;
        if (fc >= nqc) fc -= nqc;
        fill(g + 2 < total ? fc : 0, slot_t<(S + 2) % 3>());
      }
      // the chunk's fragments
      half8_t F[NDT][MT];
#pragma unroll
      for (int s = 0; s < NDT; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const uint4 v = cur[(s * MT + mt) * 64 + lane];
          F[s][mt] = *reinterpret_cast<const half8_t *>(&v);
        }
      // this lane's eight points: w z scaled, rounded in pairs
      const float *w8 = wl + qc * 32 + 8 * kb;
      float4 z0 = {1, 1, 1, 1}, z1 = {1, 1, 1, 1};
      if constexpr (COEFF) {
        z0 = *(const float4 *)(zbuf[wave] + qc * 32 + 8 * kb);
        z1 = *(const float4 *)(zbuf[wave] + qc * 32 + 8 * kb + 4);
      }
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
            acc[tile_index(I, J)] =
                __builtin_amdgcn_mfma_f32_16x16x32_f16(F[s][I], h, acc[tile_index(I, J)], 0, 0, 0);
        }
      }
      // chunk g + 1 (loaded during chunk g - 1) and the next coefficient
      // values have landed: at most the PRE direct loads of chunk g + 2 are
      // outstanding; then every wave's, at the barrier
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(PRE));
      bare_barrier();
    };
    // the cell's chunks from q0, slot of chunk qc = (PH + qc - q0) % 3
    auto chunks = [&](auto ph) {
      constexpr int PH = decltype(ph)::value;
      for (int qc = q0; qc < nqc; qc += 3) {
        step(qc, slot_t<PH>());
        if (qc + 1 < nqc) step(qc + 1, slot_t<(PH + 1) % 3>());
        if (qc + 2 < nqc) step(qc + 2, slot_t<(PH + 2) % 3>());
      }
    };
    const int ph = (g0 + q0) % 3;
    if (ph == 0) chunks(slot_t<0>());
    else if (ph == 1) chunks(slot_t<1>());
    else chunks(slot_t<2>());

    // the next cell's factors and coefficient values, then this cell's rows
    if constexpr (COEFF) {
      load_rec(ce_next, rn0, rn1);
      load_z(ce_next);
    }
    if (valid) {
      if (!COEFF && !cf.ok && lane == 0) atomicOr(a.status, STATUS_DEGENERATE);
      // the forms with fewer than 11 row tiles have n_phi a multiple of
      // four (rows of whole float4s); with 11 (n_phi = 165) the rows are
      // packed at any n_phi, and n_phi passes through an empty asm so that
      // the store offsets are formed here, per cell, instead of being kept
      // live across the walk
      constexpr bool V4_ONLY = MT < 11;
      int np = nphi;
      if constexpr (!V4_ONLY) asm volatile("" : "+s"(np));
      float *A = a.A + ce * (int64_t)np * np;  // wave-uniform
      constexpr bool v4 = V4_ONLY;
      // (at least 19 wait states between the last MFMA and the first
      // accumulator read in asm)
      if constexpr (!v4) asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7");
#pragma unroll
      for (int J = 0; J < MT; ++J) {
        // row block J: rows 16 J + x, x < 16, at rs[x n_phi + col], with rs
        // as far into the LDS buffer as the block's start is past a 16-byte
        // boundary in global memory (whole float4s on both sides)
        float *blk = A + 16 * J * np;
        float *rs = v4 ? rb : rb + (int)(((uintptr_t)blk >> 2) & 3);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
        for (int ii = 0; ii < MT; ++ii) {
          // v4: the tiles in column order, columns past n_phi skipped;
          // otherwise the last tile column first and nothing skipped: its
          // columns past n_phi run into the first columns of the next row,
          // which the later tiles overwrite (the wave's LDS writes complete
          // in order; the fence keeps the compiler from reordering them)
          const int I = v4 ? ii : ii == 0 ? MT - 1 : ii - 1;
          if (I <= J) {
            // tile (I, J): lane holds A(16 I + 4 kb + r, 16 J + c) = A(16 J + c, 16 I + 4 kb + r)
            const f32x4_t v = v4 ? acc[tile_index(I, J)] * cf.inv
                                 : agpr_tile_scaled(acc[tile_index(I, J)], cf.inv);
            const int col = 16 * I + 4 * kb;
            if (v4) {
              if (col < np) *(float4 *)(rb + c * np + col) = float4{v[0], v[1], v[2], v[3]};
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) rs[c * np + col + r] = v[r];
            }
          } else {
            // tile (J, I): lane holds A(16 J + 4 kb + r, 16 I + c)
            const f32x4_t v = v4 ? acc[tile_index(J, I)] * cf.inv
                                 : agpr_tile_scaled(acc[tile_index(J, I)], cf.inv);
            const int col = 16 * I + c;
            if (v4) {
              if (col < np)
#pragma unroll
                for (int r = 0; r < 4; ++r) rb[(4 * kb + r) * np + col] = v[r];
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) rs[(4 * kb + r) * np + col] = v[r];
            }
          }
          if (!v4 && ii == 0) __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        // (the wave's own LDS accesses complete in order; the fences keep
        // the compiler from moving them across one another)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // the block's rows (those inside the matrix) are contiguous
        const int nrow = min(16, np - 16 * J);
        if (v4) {
          const int n16 = nrow * np / 4;
          float4 *dst = (float4 *)blk;
          for (int t = lane; t < n16; t += 64) dst[t] = rbuf[wave][t];
        } else {
          // dwords up to the first 16-byte boundary, whole float4s (two
          // LDS reads ahead of their stores), then the last dwords
          const int n = nrow * np;
          const int hd = (4 - (int)(((uintptr_t)blk >> 2) & 3)) & 3;
          if (lane < hd) blk[lane] = rs[lane];
          const int nb = (n - hd) >> 2;
          const float4 *s4 = (const float4 *)(rs + hd);  // 16-byte aligned
          float4 *d4 = (float4 *)(blk + hd);               // 16-byte aligned
          int k = lane;
          for (; k + 64 < nb; k += 2 * 64) {
            const float4 w0 = s4[k], w1 = s4[k + 64];
            d4[k] = w0;
            d4[k + 64] = w1;
          }
          if (k < nb) d4[k] = s4[k];
          const int tl = hd + 4 * nb;
          if (tl + lane < n) blk[tl + lane] = rs[tl + lane];
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
    }
  }
}

template <int MT, int NDT, bool COEFF, int NW>
static fe_status launch_cellwise_one(const CellwiseLaunch &c, const CwArgs &k) {
  auto kern = cellwise_kernel<MT, NDT, COEFF, NW>;
  // dynamic: the quadrature weights (the ring and the row-block buffers are
  // static)
  const size_t smem = (size_t)c.L->n_q_pad * sizeof(float);
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
                     c.n_dofs, L.n_phi, L.n_q, L.n_q_pad, (const FormHeader *)c.form_buf, c.coords, L.d,
                     c.zpt, c.zmax, (CwRec *)c.rec, c.status);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

inline fe_status launch_cellwise(const CellwiseLaunch &c) {
  const FormLayout &L = *c.L;
  if (!cellwise_eligible(L)) return FE_EUNSUPPORTED;
  if (c.n_cells == 0) return FE_OK;
  const bool coeff = c.coeff != nullptr;
  if (coeff) {
    if (!c.zpt || !c.zmax || !c.rec) return FE_EINVAL;
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
  k.rec = coeff ? (const CwRec *)c.rec : nullptr;
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
    case 11: return launch_cellwise_one<11, 1, false, 4>(c, k);
  }
  return FE_EUNSUPPORTED;
}

}  // namespace fe
