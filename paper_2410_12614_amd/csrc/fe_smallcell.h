// Local matrices of the smallest FP16 mass forms on the vector ALUs
// (Section 3, Algorithm 1, without matrix-core tiles): P1 and P2
// tetrahedra, P1..P3 triangles (n_phi 3, 4, 6, 10).  One thread per row j of
// a local matrix: A(i, j) = sum_q B(q, i) H(q, j) for all i, with
// H(q, j) = c_K w_q B(q, j) formed as the matrix-core kernels form it (the
// cell factor c_K = sigma_K |det J_K| and the weighted table in half, their
// product rounded once to half) and products of two halves, exact in
// single, summed in single.  A workgroup takes 256 / n_phi consecutive cells
// at a time (their geometry one thread per cell), forms their rows in LDS
// and stores them as one contiguous run of 16-byte pieces.  For these forms
// the 16 x 16 tiles of the matrix cores are mostly padding (16 x 16 for a
// 4 x 4 matrix) and the kernels are bound by their per-tile overheads; here
// the whole pass is a stream of about 130 to 500 bytes per cell.
#pragma once

#include "fe_cell_kernel.h"

namespace fe {

struct SmallArgs {
  const unsigned char *afrag;  // B^T fragments (half, scaled by b_scale)
  const _Float16 *wtab;        // w_q B(q, j), [j][n_q_pad] (half, scaled by w_scale)
  const FormHeader *hdr;
  int32_t *status;
  const double *coords;
  float *A;  // [n_cells][n_phi][n_phi]
  int64_t n_cells;
  int d, n_q, n_q_pad, n_mt;
};

// Forms of this kernel: FP16 storage, simplices, the mass form without a
// coefficient, n_phi in {3, 4, 6, 10}, at most SMALL_MAX_Q points.
constexpr int SMALL_MAX_Q = 128;

template <int N>
__global__ __launch_bounds__(256) void small_cell_kernel(SmallArgs a) {
  // a workgroup pass takes CB consecutive cells: their factors (one thread
  // per cell), their rows (one thread per row), then their n_phi^2 CB
  // values, contiguous in the output, in 16-byte stores from LDS
  constexpr int CB = 256 / N;
  constexpr int NV = CB * N * N;
  __shared__ float fac[CB][2];  // per cell: c_K (a half value) and the inverse scale
  __shared__ float4 orow[(NV + 3) / 4];
  // the tables in single (exact copies of the half values): B(q, i) and
  // w_q B(q, i), [n_q][N] each
  extern __shared__ float tab[];
  float *Bt = tab, *Wt = tab + a.n_q * N;
  const int tid = threadIdx.x;
  for (int e = tid; e < a.n_q * N; e += blockDim.x) {
    const int q = e / N, i = e - q * N;
    // fragment element of B(q, i): quadrature chunk q / 32, lane
    // 16 ((q mod 32) / 8) + i mod 16, entry q mod 8
    const size_t slot = frag_slot(i / 16, 0, q / 32, a.n_mt, 1);
    const _Float16 *fr = (const _Float16 *)a.afrag;
    Bt[e] = (float)fr[(slot * 64 + ((q & 31) >> 3) * 16 + (i & 15)) * 8 + (q & 7)];
    Wt[e] = (float)a.wtab[(size_t)i * a.n_q_pad + q];
  }
  const int cl = tid / N, j = tid - cl * N;  // this thread's cell of the pass and row
  float *ov = (float *)orow;
  // 16-byte stores when a pass's values start on 16-byte boundaries
  const bool v4 = (N * N) % 4 == 0 && ((uintptr_t)a.A & 15) == 0;
  const int64_t passes = (a.n_cells + CB - 1) / CB;
  for (int64_t ps = blockIdx.x; ps < passes; ps += gridDim.x) {
    const int64_t base = ps * CB;
    const int nc = (int)min((int64_t)CB, a.n_cells - base);
    if (tid < nc) {
      // geometry (FP64, Section 4.2) and the cell factor, as in the batched
      // kernel
      const int64_t cell = base + tid;
      double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      double adet = 0.0;
      const bool ok = cell_geometry_mode(a.hdr->geom, a.d, a.coords + cell * (a.d + 1) * a.d, G, adet);
      if (!ok) atomicOr(a.status, STATUS_DEGENERATE);
      _Float16 Gp[3][3];
      float inv;
      cell_factors<PolF16>(a.hdr, 1, true, ok, G, adet, 1.0, Gp, inv);
      fac[tid][0] = (float)Gp[0][0];
      fac[tid][1] = inv;
    }
    __syncthreads();  // (the first pass: also the tables)
    if (cl < nc) {
      const float g = fac[cl][0], inv = fac[cl][1];
      float acc[N];
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = 0.0f;
      for (int q = 0; q < a.n_q; ++q) {
        // H(q, j): the product of two halves (exact in single) rounded once
        const float h = (float)(_Float16)(Wt[q * N + j] * g);
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] = fmaf(Bt[q * N + i], h, acc[i]);
      }
      // row j of the stored matrix holds sum_q B(q, i) H(q, j), as in the
      // batched kernel (a column of A_K stored as a row, by symmetry)
#pragma unroll
      for (int i = 0; i < N; ++i) ov[(cl * N + j) * N + i] = acc[i] * inv;
    }
    __syncthreads();
    // (the next pass writes orow only after the barrier that follows its
    // factors, which every thread reaches after these stores)
    const int nv = nc * N * N;
    float *dst = a.A + base * (N * N);
    if (v4) {
      for (int t = tid; t < nv / 4; t += blockDim.x) ((float4 *)dst)[t] = orow[t];
    } else {
      for (int t = tid; t < nv; t += blockDim.x) dst[t] = ov[t];
    }
  }
}

template <int N>
static fe_status launch_small_one(const SmallArgs &k, int64_t n_cells, hipStream_t s) {
  auto kern = small_cell_kernel<N>;
  const size_t smem = 2 * (size_t)k.n_q * N * sizeof(float);  // the tables (dynamic)
  LaunchInfo li;
  if (launch_info((const void *)kern, 256, smem, &li) != FE_OK) return FE_EHIP;
  const int64_t need = (n_cells + 256 / N - 1) / (256 / N);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)li.ncu * 8));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), smem, s, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

inline bool small_eligible(const FormLayout &L) {
  return L.prec == FE_FP16_ACC32 && !L.box && !L.has_coeff && L.ndt == 1 && L.n_q <= SMALL_MAX_Q &&
         (L.n_phi == 3 || L.n_phi == 4 || L.n_phi == 6 || L.n_phi == 10);
}

inline fe_status launch_small(const CellLaunch &a) {
  const FormLayout &L = *a.L;
  if (!small_eligible(L)) return FE_EUNSUPPORTED;
  if (a.n_cells == 0) return FE_OK;
  SmallArgs k;
  k.afrag = a.form_buf + L.off_afrag;
  k.wtab = (const _Float16 *)(a.form_buf + L.off_wtab);
  k.hdr = (const FormHeader *)a.form_buf;
  k.status = a.status;
  k.coords = a.coords;
  k.A = (float *)a.A_local;
  k.n_cells = a.n_cells;
  k.d = L.d;
  k.n_q = L.n_q;
  k.n_q_pad = L.n_q_pad;
  k.n_mt = L.mt;
  const hipStream_t s = (hipStream_t)a.stream;
  switch (L.n_phi) {
    case 3: return launch_small_one<3>(k, a.n_cells, s);
    case 4: return launch_small_one<4>(k, a.n_cells, s);
    case 6: return launch_small_one<6>(k, a.n_cells, s);
    case 10: return launch_small_one<10>(k, a.n_cells, s);
  }
  return FE_EUNSUPPORTED;
}

}  // namespace fe
