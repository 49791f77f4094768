// Cell kernel: local element matrices A_K = B^T H_K on the gfx950 matrix cores.
//
// Algorithm 1 (Section 3.2) with the one-H-per-s variant of the remark that
// follows it, read as H_s = sum_t C_st B_t^T, so that A = sum_s B_s H_s is a
// single contraction over K = (s, q), s < n_d.  Cells are batched 16 at a
// time (cell batching, Section 3.1) and laid along the N dimension of
// 16 x 16 x KSTEP matrix-core tiles:
//
//     [A_c(i, j)]_{i, c} = sum_k  B^T(i, k) * H_c(k, j)     for one column j,
//
// so the left operand B^T (rows i, shared by all cells) is read from the
// prepared form buffer in lane order, and the right operand (16 cells x
// KSTEP values of H for one j) is formed in registers:
//
//     H_c((s, q), j) = sigma_c z_c(X_q) sum_t G_c(s, t) (w_q B_t(q, j)),
//
// from FP64 geometry (J, det J, adj J; Section 4.2) rounded once to the
// operand format.  sigma_c = 2^e_c is an exact per-cell power of two that
// keeps H inside the FP16 range (the paper notes FP16 underflow of geometry
// terms and leaves scaling open); it is undone exactly on the FP32
// accumulator.  The left operand B^T carries its own exact power-of-two
// scale (stored in the form header) for the same reason: the matrix cores
// flush FP16 subnormal inputs.  The coefficient z at the quadrature points is the FE
// function evaluation z_q = sum_k z_k phi_k(X_q) with u_p = u^2 relative
// to the storage format: single for FP16/BF16, double for FP32, the split
// pair and FP64 (the list of precisions and the mixed-precision strategy of
// Section 4.5).
//
// Workgroup: NW waves (4, or 8 when the tables are staged in LDS).  Lane l
// of a wave owns cell c = l % 16 and K-slot kb = l / 16; wave w handles the
// columns j in [pass*NW*JC + w*JC, +JC).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fe_internal.h"

namespace fe {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
// four floats at a 4-byte aligned address (one 16-byte access in the
// target's unaligned access mode)
typedef float f4u_t __attribute__((ext_vector_type(4), aligned(4)));

// ---- precision policies -------------------------------------------------
// A/B operand layout of every 16x16 instruction used here: lane l holds
// rows/cols (l % 16) and K entries (l / 16) * KPL + e.  Output: lane l holds
// column l % 16 and rows row(l / 16, r), r < 4 (checked on gfx950).

struct PolF16 {
  static constexpr int KSTEP = 32, KPL = 8, REGMUL = 1;
  static constexpr bool SPLIT = false, SCALED = true;
  // H is computed in the storage precision (List 1: u_s stores B and C and
  // computes H): packed half FMAs on a half weighted table
  static constexpr bool H16 = true;
  typedef _Float16 hreal;
  typedef float real;
  typedef float zreal;  // coefficient evaluation: u_p = u^2 for FP16 storage
  typedef f32x4_t acc;
  typedef half8_t frag;
  static __device__ __forceinline__ frag load(const unsigned char *base, size_t idx) {
    return *(const frag *)(base + idx * 16);
  }
  static __device__ __forceinline__ frag pack(const float *h) {
    frag f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (_Float16)h[e];
    return f;
  }
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kb, int r) { return 4 * kb + r; }
};

struct PolBF16 {
  static constexpr int KSTEP = 32, KPL = 8, REGMUL = 1;
  static constexpr bool SPLIT = false, SCALED = true;
  static constexpr bool H16 = false;  // H formed in single, rounded once
  typedef float hreal;
  typedef float real;
  typedef float zreal;
  typedef f32x4_t acc;
  typedef bf16x8_t frag;
  static __device__ __forceinline__ frag load(const unsigned char *base, size_t idx) {
    return *(const frag *)(base + idx * 16);
  }
  static __device__ __forceinline__ frag pack(const float *h) {
    frag f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (__bf16)h[e];
    return f;
  }
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kb, int r) { return 4 * kb + r; }
};

// hi + 2^-11 lo pairs of halves; products hi*hi into one accumulator and
// hi*lo + lo*hi into another, combined once at the end.
struct PolSplit {
  static constexpr int KSTEP = 32, KPL = 8, REGMUL = 2;
  static constexpr bool SPLIT = true, SCALED = true;
  static constexpr bool H16 = false;  // H formed in single, then split
  typedef float hreal;
  typedef float real;
  typedef double zreal;  // the pair carries ~22 bits: u^2 calls for double
  typedef f32x4_t acc;
  typedef half8_t frag;
  static __device__ __forceinline__ frag load(const unsigned char *base, size_t idx) {
    return *(const frag *)(base + idx * 16);
  }
  static __device__ __forceinline__ void pack2(const float *h, frag &hi, frag &lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      _Float16 x = (_Float16)h[e];
      hi[e] = x;
      lo[e] = (_Float16)((h[e] - (float)x) * 2048.0f);
    }
  }
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kb, int r) { return 4 * kb + r; }
};

struct PolF32 {
  static constexpr int KSTEP = 4, KPL = 1, REGMUL = 1;
  static constexpr bool SPLIT = false, SCALED = true;
  static constexpr bool H16 = false;
  typedef float hreal;
  typedef float real;
  typedef double zreal;
  typedef f32x4_t acc;
  typedef float frag;
  static __device__ __forceinline__ frag load(const unsigned char *base, size_t idx) {
    return ((const float *)base)[idx];
  }
  static __device__ __forceinline__ frag pack(const float *h) { return h[0]; }
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kb, int r) { return 4 * kb + r; }
};

struct PolF64 {
  static constexpr int KSTEP = 4, KPL = 1, REGMUL = 2;
  static constexpr bool SPLIT = false, SCALED = false;
  static constexpr bool H16 = false;
  typedef double hreal;
  typedef double real;
  typedef double zreal;
  typedef f64x4_t acc;
  typedef double frag;
  static __device__ __forceinline__ frag load(const unsigned char *base, size_t idx) {
    return ((const double *)base)[idx];
  }
  static __device__ __forceinline__ frag pack(const double *h) { return h[0]; }
  static __device__ __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the FP64 instruction interleaves its output rows
  static __device__ __forceinline__ int row(int kb, int r) { return kb + 4 * r; }
};

// ---- kernel arguments -----------------------------------------------------
struct KArgs {
  const unsigned char *afrag;     // B^T fragments (hi for split)
  const unsigned char *afrag_lo;  // split mode
  const void *wtab;               // [NDT][n_phi][n_q_pad], P::hreal
  const void *vtab;               // [n_q][n_phi], zreal
  const FormHeader *hdr;
  int32_t *status;
  const double *coords;
  const int32_t *dofmap;
  const double *coeff;
  const double *ptab;  // hexahedra: quadrature points [n_q][3]
  int box;             // hexahedra: |det J(X_q)| per point
  void *A;
  int64_t n_cells, n_dofs;
  int d, nd, n_phi, n_q, n_q_pad, nks;
  int mt0, mt_all;     // row tiles [mt0, mt0 + MT) of the form's mt_all in this launch
};

// FP64 geometry of one affine simplex: G = |det J| J^{-1} J^{-T} computed as
// adj(J) adj(J)^T / |det J| (cofactor inverse; any inverse meeting the
// paper's inverse assumption may be used).  Returns false when det J == 0 or
// a value is not finite.
__device__ __forceinline__ bool cell_geometry(int d, const double *x, double G[3][3],
                                              double &adet) {
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) J[i][j] = x[(j + 1) * d + i] - x[i];
  double adj[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double det;
  if (d == 3) {
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
  } else {
    adj[0][0] = J[1][1];
    adj[0][1] = -J[0][1];
    adj[1][0] = -J[1][0];
    adj[1][1] = J[0][0];
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  }
  adet = fabs(det);
  const double r = 1.0 / adet;
  bool ok = (det != 0.0) && isfinite(det);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += adj[i][k] * adj[j][k];
      G[i][j] = s * r;
      ok = ok && isfinite(G[i][j]);
    }
  return ok;
}

// FP32 geometry (the geometry precision u_g = single): coordinates rounded
// to single, J, its adjugate and det J in single, G = adj adj^T / |det J|;
// also the Frobenius condition estimate ||J||_F ||adj J||_F / |det J| >=
// kappa_2(J).  Returns false when det J == 0 or a value is not finite.
__device__ __forceinline__ bool cell_geometry_f32(int d, const double *x, double G[3][3],
                                                  double &adet, float &kappa) {
  float J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) J[i][j] = (float)x[(j + 1) * d + i] - (float)x[i];
  float adj[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  float det;
  if (d == 3) {
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
  } else {
    adj[0][0] = J[1][1];
    adj[0][1] = -J[0][1];
    adj[1][0] = -J[1][0];
    adj[1][1] = J[0][0];
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  }
  const float ad = fabsf(det);
  adet = ad;
  const float r = 1.0f / ad;
  bool ok = (det != 0.0f) && isfinite(det);
  float nj = 0.0f, na = 0.0f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      nj += J[i][j] * J[i][j];
      na += adj[i][j] * adj[i][j];
      float s = 0.0f;
      for (int k = 0; k < 3; ++k) s += adj[i][k] * adj[j][k];
      G[i][j] = s * r;
      ok = ok && isfinite(G[i][j]);
    }
  kappa = sqrtf(nj) * sqrtf(na) * r;
  return ok;
}

// Above this condition estimate the AUTO geometry mode recomputes a cell in
// FP64: the single-precision error kappa u_32 then stays below 2^-14, an
// eighth of the FP16 storage unit roundoff.
constexpr float GEOM_AUTO_KAPPA = 1024.0f;

// Geometry in the precision of the form (FE_GEOM_FP64, FE_GEOM_FP32, or
// FE_GEOM_AUTO: single, and double for cells whose single-precision result
// is degenerate or whose condition estimate exceeds GEOM_AUTO_KAPPA).
__device__ __forceinline__ bool cell_geometry_mode(int mode, int d, const double *x,
                                                   double G[3][3], double &adet) {
  if (mode == FE_GEOM_FP64) return cell_geometry(d, x, G, adet);
  float kappa;
  const bool ok = cell_geometry_f32(d, x, G, adet, kappa);
  if (mode == FE_GEOM_AUTO && !(ok && kappa <= GEOM_AUTO_KAPPA)) return cell_geometry(d, x, G, adet);
  return ok;
}

// det J(X) of the trilinear map of a hexahedron with vertices x [8][3]
// (vertex v at the reference corner (v & 1, (v >> 1) & 1, (v >> 2) & 1)):
// J_ij = sum_v x_v,i d_j phi_v(X), phi_v the Q1 basis, in FP64.
__device__ __forceinline__ double box_det(const double *x, const double *X) {
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int v = 0; v < 8; ++v) {
    double f[3], df[3];
    for (int e = 0; e < 3; ++e) {
      const bool b = (v >> e) & 1;
      f[e] = b ? X[e] : 1.0 - X[e];
      df[e] = b ? 1.0 : -1.0;
    }
    const double g[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) J[i][j] += x[v * 3 + i] * g[j];
  }
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Poisson geometry tensor of the trilinear map at X, FP64:
// G = adj(J) adj(J)^T / |det J| with J_ij = sum_v x_v,i d_j phi_v(X).
// Returns false when det J == 0 or a value is not finite.
__device__ __forceinline__ bool box_poisson(const double *x, const double *X, double G[3][3]) {
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int v = 0; v < 8; ++v) {
    double f[3], df[3];
    for (int e = 0; e < 3; ++e) {
      const bool b = (v >> e) & 1;
      f[e] = b ? X[e] : 1.0 - X[e];
      df[e] = b ? 1.0 : -1.0;
    }
    const double g[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) J[i][j] += x[v * 3 + i] * g[j];
  }
  double adj[3][3];
  adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
  const double r = 1.0 / fabs(det);
  bool ok = det != 0.0 && isfinite(det);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      G[i][j] = (adj[i][0] * adj[j][0] + adj[i][1] * adj[j][1] + adj[i][2] * adj[j][2]) * r;
      ok = ok && isfinite(G[i][j]);
    }
  return ok;
}

// Unique components of a symmetric 3x3 tensor: (00, 01, 02, 11, 12, 22).
__device__ __forceinline__ int sym_comp(int s, int t) {
  const int a = s < t ? s : t, b = s < t ? t : s;
  return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

// Exact power-of-two scale exponent e of H for one cell, from a bound
// gabs >= max_s sum_t |G_st| of its geometry factors and the largest
// per-point factor zmax, and the exact inverse of all the scales (the cell's
// and those of B^T and of the half weighted table), as in cell_factors.
template <class P>
__device__ __forceinline__ int cell_scale_exp(const FormHeader *hdr, double gabs, double zmax,
                                              typename P::real &inv) {
  int esK = 0;
  if constexpr (P::H16) {
    const double bound = hdr->max_wb * hdr->w_scale * gabs * fmax(zmax, 1.0);
    if (bound > 0.0 && isfinite(bound)) esK = 14 - ilogb(bound);
  } else if constexpr (P::SCALED) {
    const double bound = hdr->max_wb * gabs * zmax;
    if (bound > 0.0 && isfinite(bound)) esK = 14 - ilogb(bound);
  }
  typedef typename P::real T;
  if constexpr (P::H16)
    inv = (T)ldexp(1.0, -esK - ilogb(hdr->b_scale) - ilogb(hdr->w_scale));
  else
    inv = (T)ldexp(1.0, -esK - ilogb(hdr->b_scale));
  return esK;
}

// Factors of H for one cell: the geometry tensor (|det J| for the mass
// form) times the exact power-of-two scale sigma = 2^e with
// |H| <= sigma max|w B| max_s sum_t |G_st| max_q |z_q| < 2^15, rounded once to
// the arithmetic type of H, and the exact inverse of sigma and of the B^T
// scale.  Invalid (padding) cells get zero factors, degenerate cells NaN.
template <class P>
__device__ __forceinline__ void cell_factors(const FormHeader *hdr, int nd, bool valid, bool ok,
                                             const double G[3][3], double adet, double zmax,
                                             typename P::hreal Gp[3][3], typename P::real &inv) {
  typedef typename P::hreal HT;
  double gabs = adet;
  if (nd > 1) {
    gabs = 0.0;
    for (int s = 0; s < 3; ++s) gabs = fmax(gabs, fabs(G[s][0]) + fabs(G[s][1]) + fabs(G[s][2]));
  }
  // half arithmetic: the partial sums over t and their product with z stay
  // below 2^15 (the table carries its own scale); all scales are exact
  // powers of two, inverted by exponents
  const double sK = ldexp(1.0, cell_scale_exp<P>(hdr, gabs, zmax, inv));
  for (int s = 0; s < 3; ++s)
    for (int t = 0; t < 3; ++t) {
      double v = (nd == 1) ? (s == 0 && t == 0 ? adet : 0.0) : G[s][t];
      if (!valid) v = 0.0;
      else if (!ok) v = NAN;
      Gp[s][t] = (HT)(v * sK);
    }
}

// H for one lane in half arithmetic: h = Gs[0] w[0] + Gs[1] w[1] + Gs[2] w[2],
// each step one packed half operation (a product, then fused multiply-adds)
// on pairs of entries; g2[t] holds Gs[t] in both halves.
template <int NDT>
__device__ __forceinline__ half8_t form_h16(const half2_t *g2, const half8_t (&w)[NDT]) {
  half8_t h;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    half2_t x = half2_t{w[0][2 * p], w[0][2 * p + 1]} * g2[0];
#pragma unroll
    for (int t = 1; t < NDT; ++t)
      x = __builtin_elementwise_fma(half2_t{w[t][2 * p], w[t][2 * p + 1]}, g2[t], x);
    h[2 * p] = x[0];
    h[2 * p + 1] = x[1];
  }
  return h;
}

// H for one lane: h[e] = sum_t Gs[t] w[t][e] (times z[e] with a coefficient),
// always summed t = 0, 1, 2 from zero so that every kernel forms the same
// values.
template <class T, int NDT, int KPL>
__device__ __forceinline__ void form_h(const T *Gs, const T (&w)[NDT][KPL], T (&h)[KPL]) {
#pragma unroll
  for (int e = 0; e < KPL; ++e) {
    T x = 0;
#pragma unroll
    for (int t = 0; t < NDT; ++t) x += Gs[t] * w[t][e];
    h[e] = x;
  }
}

// H for one lane with a geometry tensor per quadrature point (hexahedral
// Poisson form), half arithmetic: h[e] = g[0][e] w[0][e] + g[1][e] w[1][e]
// + g[2][e] w[2][e] on pairs of entries, g[t] holding G_st at this lane's
// eight points.
template <int NDT>
__device__ __forceinline__ half8_t form_h16_pp(const half8_t (&g)[NDT], const half8_t (&w)[NDT]) {
  half8_t h;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    half2_t x = half2_t{w[0][2 * p], w[0][2 * p + 1]} * half2_t{g[0][2 * p], g[0][2 * p + 1]};
#pragma unroll
    for (int t = 1; t < NDT; ++t)
      x = __builtin_elementwise_fma(half2_t{w[t][2 * p], w[t][2 * p + 1]},
                                    half2_t{g[t][2 * p], g[t][2 * p + 1]}, x);
    h[2 * p] = x[0];
    h[2 * p + 1] = x[1];
  }
  return h;
}

// The same in the arithmetic type of H (single or double), summed t = 0, 1, 2
// from zero.
template <class T, int NDT, int KPL>
__device__ __forceinline__ void form_h_pp(const T (&g)[NDT][KPL], const T (&w)[NDT][KPL],
                                          T (&h)[KPL]) {
#pragma unroll
  for (int e = 0; e < KPL; ++e) {
    T x = 0;
#pragma unroll
    for (int t = 0; t < NDT; ++t) x += g[t][e] * w[t][e];
    h[e] = x;
  }
}

// 8 (KPL = 8) or 1 consecutive entries of the weighted table
template <class T, int KPL>
__device__ __forceinline__ void load_w(const T *w, T (&v)[KPL]) {
  if constexpr (KPL == 8) {
    const float4 w0 = ((const float4 *)w)[0], w1 = ((const float4 *)w)[1];
    v[0] = w0.x; v[1] = w0.y; v[2] = w0.z; v[3] = w0.w;
    v[4] = w1.x; v[5] = w1.y; v[6] = w1.z; v[7] = w1.w;
  } else {
    v[0] = w[0];
  }
}

template <class P>
__device__ __forceinline__ typename P::frag lds_frag(const unsigned char *base, size_t idx) {
  return *(const typename P::frag *)(base + idx * sizeof(typename P::frag));
}

// Persistent cell kernel: each workgroup (NW waves) walks work items of 16
// cells (one batch, or one pass over its columns).  STAGE 1 or 2 copies the B^T fragments of the whole K range into
// LDS once; STAGE == 2 also copies the weighted table (the 16 lanes of a
// K-slot read one row j, a broadcast).  Both are then shared by all waves for
// every batch.  STAGE == 3 streams them instead: per quadrature chunk the
// fragments of the chunk (contiguous in the chunk-major layout) and the
// chunk's slice of the weighted table pass through a double-buffered LDS
// ring filled by the whole workgroup, the next chunk's loads in flight
// during the current chunk's math (forms whose tables do not fit on chip).
//
// PG (hexahedral Poisson form): the geometry tensor varies over the cell, so
// G(X_q) is evaluated in FP64 at every point of the batch's 16 cells, scaled
// by the cell's exact power of two and kept in LDS in the arithmetic type
// of H, [6 components][16 cells][n_q_pad + pad]; H is formed per point from
// it.  Row windows: a launch may cover the row tiles [mt0, mt0 + MT) of a
// form with mt_all row tiles (STAGE 0 only), for forms too wide for one.
template <class P, int MT, int JC, int NDT, bool COEFF, int STAGE, int NW, bool PG = false>
__global__ __launch_bounds__(NW * 64, 8 / NW) void cell_kernel(KArgs a) {
  typedef typename P::real T;
  typedef typename P::hreal HT;  // weighted table and H formation
  typedef typename P::zreal Z;
  typedef typename P::acc ACC;
  typedef typename P::frag FRAG;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c = lane & 15, kb = lane >> 4;
  const int d = a.d, nphi = a.n_phi, n_q_pad = a.n_q_pad, nks = a.nks;

  constexpr int NT = NW * 64;
  static_assert(STAGE != 3 || !P::SPLIT, "streamed chunks carry one fragment set");
  // STAGE 3: one ring slot = the chunk's fragments, then its table slice
  // [t][j][KSTEP]; two slots
  constexpr size_t CFRAG = (size_t)NDT * MT * 64 * sizeof(FRAG);
  const size_t ctab = (size_t)NDT * nphi * P::KSTEP * sizeof(HT);
  const size_t cslot = (CFRAG + ctab + 15) / 16 * 16;
  const size_t frag_bytes = (STAGE == 1 || STAGE == 2) ? (size_t)MT * nks * 64 * sizeof(FRAG)
                            : STAGE == 3                ? 2 * cslot
                                                        : 0;
  const size_t wtab_bytes = STAGE == 2 ? (size_t)NDT * nphi * n_q_pad * sizeof(HT) : 0;
  unsigned char *s_af = smem;
  unsigned char *s_afl = smem + frag_bytes;
  HT *s_wt = (HT *)(smem + frag_bytes * (P::SPLIT ? 2 : 1));
  unsigned char *zbase = smem + frag_bytes * (P::SPLIT ? 2 : 1) + wtab_bytes;
  // per-point factors z_q: the coefficient, times |det J(X_q)| for the
  // hexahedral mass form (none for the hexahedral Poisson form without a
  // coefficient: its per-point geometry is in gq)
  const int zq_len = (a.coeff || (a.box && !PG)) ? n_q_pad : 0;
  Z *zq = (Z *)zbase;                                                   // [zq_len][16]
  // [16][24] vertex coordinates of hexahedra, then [16][n_phi] coefficient dofs
  double *zloc = (double *)(zbase + (size_t)16 * zq_len * sizeof(Z));
  const int zoff = a.box ? 16 * 24 : 0;
  double *zred = zloc + zoff + (a.coeff ? 16 * nphi : 0);  // [NT]
  constexpr int GPAD = 16 / (int)sizeof(HT);
  const int gstride = n_q_pad + GPAD;
  HT *gq = (HT *)(zred + NT);  // PG: [6][16][gstride]

  if constexpr (STAGE == 1 || STAGE == 2) {
    const size_t n16 = frag_bytes / 16;
    const uint4 *src = (const uint4 *)a.afrag;
    uint4 *dst = (uint4 *)s_af;
    for (size_t t = tid; t < n16; t += NT) dst[t] = src[t];
    if constexpr (P::SPLIT) {
      const uint4 *src2 = (const uint4 *)a.afrag_lo;
      uint4 *dst2 = (uint4 *)s_afl;
      for (size_t t = tid; t < n16; t += NT) dst2[t] = src2[t];
    }
  }
  if constexpr (STAGE == 2) {
    const size_t n16 = wtab_bytes / 16;
    for (size_t t = tid; t < n16; t += NT) ((uint4 *)s_wt)[t] = ((const uint4 *)a.wtab)[t];
  }
  if constexpr (STAGE == 1 || STAGE == 2) __syncthreads();
  // STAGE 3: copy quadrature chunk qc into ring slot `slot` (all threads),
  // through registers so that the loads can be issued early
  // (n_phi <= 16 MT bounds the table slice of a chunk)
  constexpr int PRE =
      STAGE == 3 ? (int)((CFRAG + (size_t)NDT * 16 * MT * P::KSTEP * sizeof(HT)) / 16 + NT - 1) / NT
                 : 1;
  const int c16 = (int)(CFRAG / 16), t16 = (int)(ctab / 16), n16c = c16 + t16;
  const int trow16 = P::KSTEP * (int)sizeof(HT) / 16;  // 16-byte pieces per table row slice
  auto chunk_src = [&](int qc, int e) -> const uint4 * {
    if (e < c16) return (const uint4 *)(a.afrag + (size_t)qc * CFRAG) + e;
    const int r = (e - c16) / trow16, piece = (e - c16) - r * trow16;  // row r = t * nphi + j
    return (const uint4 *)((const HT *)a.wtab + (size_t)r * n_q_pad + (size_t)qc * P::KSTEP) +
           piece;
  };

  // Work items: without a coefficient one (batch of 16 cells, pass over
  // NW * JC columns) per item, so that large forms spread evenly over the
  // workgroups; with one, a whole batch (its coefficient values at the
  // quadrature points are shared by the passes).
  const int64_t nbatch = (a.n_cells + 15) / 16;
  const int npass = (nphi + NW * JC - 1) / (NW * JC);
  const int64_t nitems = COEFF ? nbatch : nbatch * npass;
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int64_t batch = COEFF ? item : item / npass;
    const int pass_lo = COEFF ? 0 : (int)(item - batch * npass);
    const int pass_hi = COEFF ? npass : pass_lo + 1;
    const int64_t cell0 = batch * 16;
    const int64_t cell = cell0 + c;
    const bool valid = cell < a.n_cells;

    // ---- geometry (Section 4.2), one lane per cell, FP64 ----
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double adet = 0.0;
    bool ok = true;
    if (a.box) {
      adet = 1.0;  // hexahedra: |det J| varies over the cell; it enters per point below
    } else if (valid) {
      ok = cell_geometry_mode(a.hdr->geom, d, a.coords + cell * (d + 1) * d, G, adet);
    }

    // ---- coefficient at the quadrature points (FE function evaluation) ----
    double zmax = 1.0;
    // Per-point factor z_q of H: the coefficient at the point, times
    // |det J(X_q)| for hexahedra (the trilinear map's Jacobian varies over
    // the cell; Section 3.1 with G(X) = |det J(X)| for the mass form).
    if constexpr (COEFF) {
      __syncthreads();  // the previous batch is done with zq
      if (a.box)
        for (int idx = tid; idx < 16 * 24; idx += NT) {
          const int64_t ce = cell0 + idx / 24;
          zloc[idx] = ce < a.n_cells ? a.coords[ce * 24 + idx % 24] : 0.0;
        }
      if (a.coeff)
        for (int idx = tid; idx < 16 * nphi; idx += NT) {
          const int cc = idx / nphi, k = idx - cc * nphi;
          const int64_t ce = cell0 + cc;
          double z = 0.0;
          if (ce < a.n_cells) {
            const int32_t g = a.dofmap[ce * nphi + k];
            if (g >= 0 && g < a.n_dofs) z = a.coeff[g];
            else atomicOr(a.status, STATUS_BAD_DOF);
          }
          zloc[zoff + idx] = z;
        }
      __syncthreads();
      const Z *vt = (const Z *)a.vtab;
      double zpart = 0.0;  // this thread's |z_q| maximum for cell tid % 16
      for (int idx = tid; idx < 16 * zq_len; idx += NT) {
        const int q = idx >> 4, cc = idx & 15;
        Z z = 0;
        if (q < a.n_q) {
          if (a.coeff) {
            for (int k = 0; k < nphi; ++k) z += (Z)zloc[zoff + cc * nphi + k] * vt[q * nphi + k];
          } else {
            z = 1;
          }
          if (!PG && a.box && cell0 + cc < a.n_cells) {
            const double dj = box_det(zloc + cc * 24, a.ptab + 3 * q);
            if (!(dj != 0.0 && isfinite(dj))) {
              atomicOr(a.status, STATUS_DEGENERATE);
              z = (Z)NAN;
            } else {
              z = z * (Z)fabs(dj);
            }
          }
        }
        zq[idx] = z;
        zpart = fmax(zpart, fabs((double)z));
      }
      zred[tid] = zpart;
      __syncthreads();
      // max_q |z_q| of this lane's cell (threads tid and tid + 16 r share tid % 16)
      double m = 0.0;
      for (int r = 0; r < NT / 16; ++r) m = fmax(m, zred[c + 16 * r]);
      zmax = zq_len > 0 ? m : 1.0;
    }
    // the per-point factors of this lane's cell enter H scaled by the exact
    // power of two zs that brings max_q |z_q| into [1, 2) (per-point |det J|
    // of a small hexahedron would otherwise be subnormal in half); the
    // inverse goes into the cell's exact inverse scale below
    int ez = 0;
    if constexpr (COEFF) {
      if (zmax > 0.0 && isfinite(zmax)) {
        ez = ilogb(zmax);
        zmax = ldexp(zmax, -ez);
      }
    }
    const T zs = (T)ldexp(1.0, -ez);

    if (valid && !ok && wave == 0 && kb == 0) atomicOr(a.status, STATUS_DEGENERATE);
    HT Gp[3][3];
    T inv;
    cell_factors<P>(a.hdr, a.nd, valid, ok, G, adet, zmax, Gp, inv);
    if constexpr (PG) {
      // G(X_q) of the batch's cells (thread tid works on cell tid % 16 = c,
      // as NT is a multiple of 16): first the bound max_q max_s sum_t
      // |G_st(X_q)| of each cell for its scale, then the scaled values
      double gpart = 0.0;
      bool okp = true;
      for (int idx = tid; idx < 16 * a.n_q; idx += NT) {
        const int q = idx >> 4, cc = idx & 15;
        if (cell0 + cc < a.n_cells) {
          double Gq[3][3];
          if (box_poisson(zloc + cc * 24, a.ptab + 3 * q, Gq)) {
            for (int s2 = 0; s2 < 3; ++s2)
              gpart = fmax(gpart, fabs(Gq[s2][0]) + fabs(Gq[s2][1]) + fabs(Gq[s2][2]));
          } else {
            okp = false;
          }
        }
      }
      __syncthreads();  // every thread has read zred for zmax
      zred[tid] = okp ? gpart : -1.0;
      __syncthreads();
      double gm = 0.0;
      bool okc = true;
      for (int r = 0; r < NT / 16; ++r) {
        const double v = zred[c + 16 * r];
        okc = okc && v >= 0.0;
        gm = fmax(gm, v);
      }
      const double sK = ldexp(1.0, cell_scale_exp<P>(a.hdr, gm, zmax, inv));
      for (int idx = tid; idx < 16 * n_q_pad; idx += NT) {
        const int q = idx >> 4, cc = idx & 15;
        const bool live = cell0 + cc < a.n_cells && q < a.n_q;
        double Gq[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (live) box_poisson(zloc + cc * 24, a.ptab + 3 * q, Gq);
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2)
#pragma unroll
          for (int t2 = s2; t2 < 3; ++t2) {
            const double v = live ? (okc ? Gq[s2][t2] * sK : NAN) : 0.0;
            gq[((size_t)sym_comp(s2, t2) * 16 + cc) * gstride + q] = (HT)v;
          }
      }
      if (valid && !okc && wave == 0 && kb == 0) atomicOr(a.status, STATUS_DEGENERATE);
      __syncthreads();
    }
    inv = (T)ldexp((double)inv, ez);

    const HT *wt = (const HT *)a.wtab;
    for (int pass = pass_lo; pass < pass_hi; ++pass) {
      const int jb = pass * NW * JC + wave * JC;
      if (STAGE != 3 && jb >= nphi) continue;
      const bool active = jb < nphi;
      ACC acc[MT][JC];
      ACC acc2[P::SPLIT ? MT : 1][P::SPLIT ? JC : 1];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
          acc[mt][jj] = ACC{0, 0, 0, 0};
          if constexpr (P::SPLIT) acc2[mt][jj] = ACC{0, 0, 0, 0};
        }
      // K = (s, q) is walked as q-chunk outer, s inner: one chunk of the
      // weighted table serves all s, and the accumulation order of every
      // output is (chunk 0: s = 0..NDT-1), (chunk 1: ...), as in the fused
      // kernel.
      const int nqc = n_q_pad / P::KSTEP;
      if constexpr (STAGE == 3) {
        for (int e = tid; e < n16c; e += NT) ((uint4 *)s_af)[e] = *chunk_src(0, e);
        __syncthreads();
      }
      for (int qc = 0; qc < nqc; ++qc) {
        const int qb = qc * P::KSTEP + kb * P::KPL;
        uint4 pre[PRE];
        unsigned char *slot = s_af + (size_t)(qc & 1) * cslot;
        if constexpr (STAGE == 3) {
          if (qc + 1 < nqc) {
#pragma unroll
            for (int p = 0; p < PRE; ++p) {
              const int e = tid + p * NT;
              if (e < n16c) pre[p] = *chunk_src(qc + 1, e);
            }
          }
        }
        FRAG afr[NDT][MT];
        FRAG afl[P::SPLIT ? NDT : 1][P::SPLIT ? MT : 1];
#pragma unroll
        for (int s = 0; s < NDT; ++s)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const size_t fi = frag_slot(a.mt0 + mt, s, qc, a.mt_all, NDT) * 64 + lane;
            if constexpr (STAGE == 3) {
              afr[s][mt] = lds_frag<P>(slot, ((size_t)s * MT + mt) * 64 + lane);
            } else if constexpr (STAGE >= 1) {
              afr[s][mt] = lds_frag<P>(s_af, fi);
              if constexpr (P::SPLIT) afl[s][mt] = lds_frag<P>(s_afl, fi);
            } else {
              afr[s][mt] = P::load(a.afrag, fi);
              if constexpr (P::SPLIT) afl[s][mt] = P::load(a.afrag_lo, fi);
            }
          }
        T zf[P::KPL];
        // without PG every coefficient-path form has per-point factors; the
        // test is then a compile-time one, so that H and its rounding to the
        // operand format compile exactly as in the fused kernel (same bits)
        const bool zmul = PG ? a.coeff != nullptr : COEFF;
        if (zmul) {
#pragma unroll
          for (int e = 0; e < P::KPL; ++e) zf[e] = (T)zq[(qb + e) * 16 + c] * zs;
        }
        // PG: the six components of G at this lane's points
        typedef typename std::conditional<P::H16, half8_t, HT[P::KPL]>::type GV;
        GV gv[PG ? 6 : 1];
        if constexpr (PG) {
#pragma unroll
          for (int cp = 0; cp < 6; ++cp) {
            const HT *src = gq + ((size_t)cp * 16 + c) * gstride + qb;
            if constexpr (P::H16) gv[cp] = *(const half8_t *)src;
            else load_w<HT, P::KPL>(src, gv[cp]);
          }
        }
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
          if (STAGE == 3 && !active) break;
          const int jl = min(jb + jj, nphi - 1);
          // row stride of the table between derivative slabs t, and the
          // start of row jl at this lane's K entries
          const size_t tstride = STAGE == 3 ? (size_t)nphi * P::KSTEP : (size_t)nphi * n_q_pad;
          const HT *wj = STAGE == 3 ? (const HT *)(slot + CFRAG) + (size_t)jl * P::KSTEP + kb * P::KPL
                         : (STAGE == 2 ? s_wt : wt) + (size_t)jl * n_q_pad + qb;
          if constexpr (P::H16) {
            half8_t wv[NDT];
#pragma unroll
            for (int t = 0; t < NDT; ++t) wv[t] = *(const half8_t *)(wj + (size_t)t * tstride);
#pragma unroll
            for (int s = 0; s < NDT; ++s) {
              half8_t hf;
              if constexpr (PG) {
                half8_t g8[NDT];
#pragma unroll
                for (int t = 0; t < NDT; ++t) g8[t] = gv[sym_comp(s, t)];
                hf = form_h16_pp<NDT>(g8, wv);
              } else {
                half2_t g2[NDT];
#pragma unroll
                for (int t = 0; t < NDT; ++t) g2[t] = half2_t{Gp[s][t], Gp[s][t]};
                hf = form_h16<NDT>(g2, wv);
              }
              if (zmul) {
                half8_t z8;
#pragma unroll
                for (int e = 0; e < 8; ++e) z8[e] = (_Float16)zf[e];
                hf = hf * z8;
              }
#pragma unroll
              for (int mt = 0; mt < MT; ++mt) acc[mt][jj] = P::mma(afr[s][mt], hf, acc[mt][jj]);
            }
          } else {
            T wv[NDT][P::KPL];
#pragma unroll
            for (int t = 0; t < NDT; ++t) load_w<T, P::KPL>(wj + (size_t)t * tstride, wv[t]);
#pragma unroll
            for (int s = 0; s < NDT; ++s) {
              T h[P::KPL];
              if constexpr (PG) {
                T g8[NDT][P::KPL];
#pragma unroll
                for (int t = 0; t < NDT; ++t)
#pragma unroll
                  for (int e = 0; e < P::KPL; ++e) g8[t][e] = gv[sym_comp(s, t)][e];
                form_h_pp<T, NDT, P::KPL>(g8, wv, h);
              } else {
                form_h<T, NDT, P::KPL>(Gp[s], wv, h);
              }
              if (zmul) {
#pragma unroll
                for (int e = 0; e < P::KPL; ++e) h[e] *= zf[e];
              }
              if constexpr (P::SPLIT) {
                FRAG hh, hl;
                P::pack2(h, hh, hl);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                  acc[mt][jj] = P::mma(afr[s][mt], hh, acc[mt][jj]);
                  acc2[mt][jj] = P::mma(afr[s][mt], hl, acc2[mt][jj]);
                  acc2[mt][jj] = P::mma(afl[s][mt], hh, acc2[mt][jj]);
                }
              } else {
                const FRAG hf = P::pack(h);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][jj] = P::mma(afr[s][mt], hf, acc[mt][jj]);
              }
            }
          }
        }
        if constexpr (STAGE == 3) {
          // the other ring slot was last read in chunk qc - 1, which every
          // wave finished before the barrier closing that chunk
          if (qc + 1 < nqc) {
            uint4 *dst = (uint4 *)(s_af + (size_t)((qc + 1) & 1) * cslot);
#pragma unroll
            for (int p = 0; p < PRE; ++p) {
              const int e = tid + p * NT;
              if (e < n16c) dst[e] = pre[p];
            }
          }
          __syncthreads();
        }
      }
      // The tile holds column j of A_K (rows i); by the symmetry of the mass
      // and stiffness forms it is stored as row j, so each lane's rows land
      // on consecutive addresses: with single-precision outputs (rows 4 kb + r)
      // a lane's four values are one 16-byte store (4-byte aligned: the
      // target's unaligned access mode), the row tail element by element.
      if (valid && active) {
        T *A = (T *)a.A + (size_t)cell * nphi * nphi;
        // row by row: consecutive stores of a lane fill consecutive addresses
#pragma unroll
        for (int jj = 0; jj < JC; ++jj)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            const int j = jb + jj;
            if (j < nphi) {
              T v[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                v[r] = acc[mt][jj][r];
                if constexpr (P::SPLIT) v[r] += acc2[mt][jj][r] * (T)(1.0 / 2048.0);
                v[r] *= inv;
              }
              const int i_base = (a.mt0 + mt) * 16;
              T *dst = A + (size_t)j * nphi + i_base;
              if constexpr (sizeof(T) == 4) {
                const int i0 = 4 * kb;  // P::row(kb, r) = 4 kb + r
                if (i_base + i0 + 3 < nphi) {
                  *(f4u_t *)(dst + i0) = f4u_t{v[0], v[1], v[2], v[3]};
                  continue;
                }
              }
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (i_base + P::row(kb, r) < nphi) dst[P::row(kb, r)] = v[r];
            }
          }
      }
    }
  }
}

template <class P, int MT, int JC, int NDT, bool COEFF, int STAGE, int NW, bool PG = false>
static fe_status launch_one(const KArgs &k, int64_t n_cells, size_t smem, int occ, hipStream_t s) {
  auto kern = cell_kernel<P, MT, JC, NDT, COEFF, STAGE, NW, PG>;
  LaunchInfo li;
  if (launch_info((const void *)kern, NW * 64, smem, &li) != FE_OK) return FE_EHIP;
  const int ncu = li.ncu;
  // work items as in the kernel: (batch, pass) without a coefficient
  const int64_t nbatch = (n_cells + 15) / 16;
  const int64_t nitems = COEFF ? nbatch : nbatch * ((k.n_phi + NW * JC - 1) / (NW * JC));
  // eight waves per compute unit: two 4-wave or one 8-wave workgroup (occ
  // doubles the workgroups; those the LDS cannot hold wait for a slot)
  const int per_cu = ((NW == 4 && smem <= 80 * 1024) ? 2 : 1) << occ;
  const int64_t blocks = std::min<int64_t>(nitems, (int64_t)ncu * per_cu);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), smem, s, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

template <class P, int MT, int JC, int NW, int STAGE>
static fe_status launch_mt(const KArgs &k, int64_t n_cells, size_t smem, int occ, hipStream_t s,
                           int ndt, bool coeff) {
  if (ndt == 1)
    return coeff ? launch_one<P, MT, JC, 1, true, STAGE, NW>(k, n_cells, smem, occ, s)
                 : launch_one<P, MT, JC, 1, false, STAGE, NW>(k, n_cells, smem, occ, s);
  return coeff ? launch_one<P, MT, JC, 3, true, STAGE, NW>(k, n_cells, smem, occ, s)
               : launch_one<P, MT, JC, 3, false, STAGE, NW>(k, n_cells, smem, occ, s);
}

// Hexahedral forms in row windows of at most 8 row tiles (one launch per
// window, each forming H again): 4-wave workgroups reading the fragments and
// the weighted table through the caches (variant 2), per-point factors in
// LDS; the Poisson form (PG) keeps G(X_q) per point there too.
template <class P, int MT, bool PG>
static fe_status launch_window(KArgs k, int64_t n_cells, size_t smem, int occ, hipStream_t s) {
  // columns per wave: the accumulators, the fragments of three slabs and the
  // per-point tensor fit the registers of two waves per SIMD
  constexpr int JC = PG ? (MT == 8 ? 2 : (MT == 6 ? 3 : 4))
                        : (P::REGMUL == 1 ? (MT == 8 ? 4 : (MT == 6 ? 7 : (MT == 4 ? 7 : (MT == 2 ? 8 : 4))))
                                          : (MT == 8 ? 2 : (MT == 6 ? 3 : (MT == 2 ? 5 : 4))));
  constexpr int NDT = PG ? 3 : 1;
  return launch_one<P, MT, JC, NDT, true, 0, 4, PG>(k, n_cells, smem, occ, s);
}

template <class P, bool PG>
static fe_status launch_box(const CellLaunch &a, KArgs k, int occ) {
  const FormLayout &L = *a.L;
  typedef typename P::hreal HT;
  const size_t zq = (L.has_coeff || !PG) ? (size_t)16 * L.n_q_pad * sizeof(typename P::zreal) : 0;
  const size_t zl = (size_t)(L.has_coeff ? L.n_phi : 0) + 24;
  const size_t gq = PG ? (size_t)6 * 16 * (L.n_q_pad + 16 / sizeof(HT)) * sizeof(HT) : 0;
  const size_t smem = zq + (size_t)16 * zl * 8 + 256 * 8 + gq;
  if (smem > 156 * 1024) return FE_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)a.stream;
  k.mt_all = L.mt;
  for (int mt0 = 0; mt0 < L.mt; mt0 += 8) {
    const int w = std::min(8, L.mt - mt0);
    k.mt0 = mt0;
    fe_status st = FE_EUNSUPPORTED;
    switch (w) {
      case 1: st = launch_window<P, 1, PG>(k, a.n_cells, smem, occ, s); break;
      case 2: st = launch_window<P, 2, PG>(k, a.n_cells, smem, occ, s); break;
      case 4: st = launch_window<P, 4, PG>(k, a.n_cells, smem, occ, s); break;
      case 6: st = launch_window<P, 6, PG>(k, a.n_cells, smem, occ, s); break;
      case 8: st = launch_window<P, 8, PG>(k, a.n_cells, smem, occ, s); break;
      default: break;
    }
    if (st != FE_OK) return st;
  }
  return FE_OK;
}

template <class P>
fe_status launch_cell_impl(const CellLaunch &a) {
  const FormLayout &L = *a.L;
  int mt, jc;
  tile_choice(L.n_phi, P::REGMUL, &mt, &jc);
  // with per-point factors (their registers and the factor reads) 6 columns
  // of 8 row tiles spill; 4 columns cover n_phi <= 128 in 8 passes.  A
  // weighted stiffness form at 6 row tiles (P6) spills with 7 columns and
  // runs 1.5x faster with 3 (84 columns in 7 passes of 12)
  if ((L.has_coeff || L.box) && mt == 8 && jc == 6) jc = 4;
  if (L.has_coeff && L.ndt == 3 && mt == 6 && jc == 7) jc = 3;
  KArgs k;
  k.afrag = a.form_buf + L.off_afrag;
  k.afrag_lo = a.form_buf + L.off_afrag_lo;
  k.wtab = a.form_buf + L.off_wtab;
  k.vtab = a.form_buf + L.off_vtab;
  k.hdr = (const FormHeader *)a.form_buf;
  k.status = a.status;
  k.coords = a.coords;
  k.dofmap = a.dofmap;
  k.coeff = a.coeff;
  k.box = L.box;
  k.ptab = (const double *)(a.form_buf + L.off_ptab);
  k.A = a.A_local;
  k.n_cells = a.n_cells;
  k.n_dofs = a.n_dofs;
  k.d = L.d;
  k.nd = L.nd;
  k.n_phi = L.n_phi;
  k.n_q = L.n_q;
  k.n_q_pad = L.n_q_pad;
  k.nks = L.nks;
  k.mt0 = 0;
  k.mt_all = L.mt;
  // Hexahedra of the Poisson form (per-point G) and forms wider than 11 row
  // tiles (Q5..Q7: 14, 22, 32) run in row windows through the caches
  if (L.box && (L.ndt == 3 || L.mt > 8)) {
    if (a.tile >= 0 && a.tile % 4 != 2) return FE_EUNSUPPORTED;
    const int occ = a.tile < 0 ? 0 : a.tile / 4;
    if (occ > 1) return FE_EINVAL;
    return L.ndt == 3 ? launch_box<P, true>(a, k, occ) : launch_box<P, false>(a, k, occ);
  }
  // per-point factors of H: a coefficient, or |det J(X_q)| of hexahedra
  const bool coeff = L.has_coeff != 0 || L.box != 0;
  const size_t zl = (size_t)(L.has_coeff ? L.n_phi : 0) + (L.box ? 24 : 0);
  typedef typename P::frag FRAG;
  typedef typename P::real T;
  const size_t frag_bytes = (size_t)mt * L.nks * 64 * sizeof(FRAG) * (P::SPLIT ? 2 : 1);
  const size_t wtab_bytes = (size_t)L.ndt * L.n_phi * L.n_q_pad * sizeof(typename P::hreal);
  hipStream_t s = (hipStream_t)a.stream;
  const int ndt = L.ndt;
  // Tile variants (CellLaunch::tile = variant + 4 occ):
  //   0: 8-wave workgroups, fragments and weighted table in LDS (small forms:
  //      row tiles <= 4, both fit)
  //   1: 4-wave workgroups, fragments in LDS (they fit beside the
  //      coefficient tables)
  //   2: 4-wave workgroups, fragments and table read through the caches
  //   3: 8-wave workgroups, fragments and table streamed through LDS one
  //      quadrature chunk at a time (not for the split mode)
  // occ = 1 launches twice the workgroups per compute unit.  The default
  // (tile < 0) is the first variant that applies, occ = 0.  Every variant
  // sums each entry in the same order, so all give identical results.
  const size_t zbytes8 = coeff ? (size_t)16 * L.n_q_pad * sizeof(typename P::zreal) +
                                     (size_t)16 * zl * 8 + 512 * 8
                               : 0;
  const size_t smem8 = frag_bytes + wtab_bytes + zbytes8;
  const size_t zbytes = coeff ? (size_t)16 * L.n_q_pad * sizeof(typename P::zreal) +
                                    (size_t)16 * zl * 8 + 256 * 8
                              : 0;
  const size_t cslot = ((size_t)ndt * mt * 64 * sizeof(FRAG) +
                         (size_t)ndt * L.n_phi * P::KSTEP * sizeof(typename P::hreal) + 15) /
                        16 * 16;
  const size_t smem3 = 2 * cslot + zbytes8;
  const bool ok8 = mt <= 4 && smem8 <= 156 * 1024;
  const bool ok1 = frag_bytes + zbytes <= 80 * 1024;
  const bool ok3 = !P::SPLIT && smem3 <= 156 * 1024;
  int variant = ok8 ? 0 : (ok1 ? 1 : 2), occ = 0;
  if (a.tile >= 0) {
    variant = a.tile % 4;
    occ = a.tile / 4;
    if (occ > 1) return FE_EINVAL;
    if ((variant == 0 && !ok8) || (variant == 1 && !ok1) || (variant == 3 && !ok3))
      return FE_EUNSUPPORTED;
  }
  if (variant == 0) {
    int jc8 = 0;
    if (mt == 1) jc8 = 2;
    if (mt == 2) jc8 = 4;
    if (mt == 3) jc8 = 5;
    if (mt == 4) jc8 = (P::REGMUL == 1) ? 7 : 4;
#define FE_C8(M, J) \
  if (mt == M && jc8 == J) return launch_mt<P, M, J, 8, 2>(k, a.n_cells, smem8, occ, s, ndt, coeff);
    FE_C8(1, 2) FE_C8(2, 4) FE_C8(3, 5) FE_C8(4, 7) FE_C8(4, 4)
#undef FE_C8
    return FE_EUNSUPPORTED;
  }
  const bool stage = variant == 1;
  const size_t smem = (stage ? frag_bytes : 0) + zbytes;
  if (variant == 3) {
    // columns per wave: as the 4-wave tiles, fewer where their accumulators
    // would not fit the registers of two waves per SIMD
    if constexpr (!P::SPLIT) {
#define FE_CASE3(M, J) \
  if (mt == M) return launch_mt<P, M, J, 8, 3>(k, a.n_cells, smem3, occ, s, ndt, coeff);
      if constexpr (P::REGMUL == 1) {
        FE_CASE3(1, 4) FE_CASE3(2, 8) FE_CASE3(3, 9) FE_CASE3(4, 7) FE_CASE3(6, 7) FE_CASE3(8, 4)
        FE_CASE3(11, 3)
      } else {
        FE_CASE3(1, 4) FE_CASE3(2, 5) FE_CASE3(3, 5) FE_CASE3(4, 4) FE_CASE3(6, 3) FE_CASE3(8, 2)
        FE_CASE3(11, 2)
      }
#undef FE_CASE3
    }
    return FE_EUNSUPPORTED;
  }
#define FE_CASE(M, J)                                                                        \
  if (mt == M && jc == J) {                                                                  \
    if (stage) return launch_mt<P, M, J, 4, 1>(k, a.n_cells, smem, occ, s, ndt, coeff);      \
    return launch_mt<P, M, J, 4, 0>(k, a.n_cells, smem, occ, s, ndt, coeff);                 \
  }
  if constexpr (P::REGMUL == 1) {
    FE_CASE(1, 4) FE_CASE(2, 8) FE_CASE(3, 9) FE_CASE(4, 7) FE_CASE(6, 7) FE_CASE(8, 6)
    FE_CASE(6, 3) FE_CASE(8, 4) FE_CASE(11, 3)
  } else {
    FE_CASE(1, 4) FE_CASE(2, 5) FE_CASE(3, 5) FE_CASE(4, 4) FE_CASE(6, 3) FE_CASE(8, 2)
    FE_CASE(11, 2)
  }
#undef FE_CASE
  return FE_EUNSUPPORTED;
}

}  // namespace fe
