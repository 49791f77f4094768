// Action kernels: Algorithm 2 of Croci & Wells (Section 3.2) for the mass
// and Poisson forms with an optional coefficient z, batched over cells as in
// Section 3.1 (V = sum_s B_s R_s with the cells of a batch as columns), and
// the adjoint density of the coefficient.
//
// For each cell K and quadrature point X_q (affine cells: G constant):
//   evaluation   x_t(q) = sum_k x_k T_t(q, k)            (gradient slabs t, or
//                                                        values for mass)
//                z(q)   = sum_k z_k phi_k(X_q)
//   step 2       r_s(q) = w_q z(q) (G grad x)_s          (w_q z(q) |det J| x(q))
//   step 3       v_i    = sum_s sum_q B_s(i, q) r_s(q)
//   adjoint      g_i    = sum_q phi_i(X_q) w_q (grad y)^T G (grad x)
//                         (w_q |det J| y(q) x(q) for mass), y a second function
//
// Layout on the matrix cores (16x16x4 instructions of the arithmetic type):
// a wave owns 16 cells, one per column (N).  Evaluation multiplies the
// table T_t (16 quadrature rows x 4 dofs per K-step) by the cells' dofs held
// in registers (lane l: cell l % 16, dof 4 ks + l / 16); its output leaves
// lane l the points q = row(l / 16, r), r < 4, of cell l % 16 -- exactly the
// B operand the contraction with B_s (M = dofs i, K = those 4 points per
// instruction r) needs, so r_s is formed in registers and never leaves the
// lane.  The tables of one tile of 16 points (evaluation, contraction and
// weights; see FormLayout::act) are staged in LDS for all waves of the
// workgroup, double buffered, when staging is enabled, else read from L2.
#pragma once

#include <hip/hip_runtime.h>

#include "fe_cell_kernel.h"

namespace fe {

struct ActArgs {
  const unsigned char *chunks;  // form_buf + off_act
  const double *coords;
  const int32_t *dofmap;
  const double *coeff;
  const void *x0, *x1;
  void *out0, *out1;
  int32_t *status;
  int64_t n_cells, n_dofs;
  int d, n_phi, nks, mt, nqt, nt;
  int geom;      // geometry precision (FE_GEOM_*)
  size_t chunk;  // elements per tile chunk
};

template <class T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
};
template <>
struct Vec16<double> {
  typedef double2 type;
};

// KS: K-steps of 4 dofs held per lane (the table's padded count, so that
// every instruction of the tile loops is unconditional); MT = ceil(KS / 4)
// row tiles; STIFF: Poisson form (gradients; triangles carry a zero third
// slab) else mass (values); COEFF: coefficient z; GZ: the adjoint density
// with the second function x1; STAGE: LDS staging of the tables.
template <class P, int KS, bool STIFF, bool COEFF, bool GZ, bool STAGE, int NW>
__global__ __launch_bounds__(NW * 64) void action_kernel(ActArgs a) {
  typedef typename P::real T;
  typedef typename P::acc ACC;
  typedef typename Vec16<T>::type V16;
  constexpr int MT = (KS + 3) / 4;
  constexpr int NE = STIFF ? 3 : 1;  // evaluated components per function
  constexpr int NT = STIFF ? 4 : 1;  // tables: values (+ three gradient slabs)
  constexpr int EPV = 16 / sizeof(T);
  constexpr int C_OFF = NT * KS * 64, W_OFF = C_OFF + NT * MT * 4 * 64;
  constexpr int CHUNK = W_OFF + 64;
  constexpr int NVEC = CHUNK / EPV;
  constexpr int PMAX = (NVEC + NW * 64 - 1) / (NW * 64);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c = lane & 15, kb = lane >> 4;
  const int d = a.d, n_phi = a.n_phi;
  const T *gch = (const T *)a.chunks;
  constexpr size_t chunk = CHUNK;
  constexpr int nvec = NVEC;
  T *lbuf = (T *)smem;
  const int64_t n_batches = (a.n_cells + 15) / 16;

  for (int64_t g0 = (int64_t)blockIdx.x * NW; g0 < n_batches; g0 += (int64_t)gridDim.x * NW) {
    const int64_t cell = (g0 + wave) * 16 + c;
    const bool valid = cell < a.n_cells;
    // the cell's dofs as B operands: K-step ks holds dof 4 ks + kb
    T X0[KS], X1[GZ ? KS : 1], Zk[COEFF ? KS : 1];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      X0[ks] = 0;
      if constexpr (GZ) X1[ks] = 0;
      if constexpr (COEFF) Zk[ks] = 0;
      const int k = 4 * ks + kb;
      if (valid && k < n_phi) {
        const int32_t dof = a.dofmap[cell * n_phi + k];
        if (dof >= 0 && dof < a.n_dofs) {
          X0[ks] = ((const T *)a.x0)[dof];
          if constexpr (GZ) X1[ks] = ((const T *)a.x1)[dof];
          if constexpr (COEFF) Zk[ks] = (T)a.coeff[dof];
        } else {
          atomicOr(a.status, (int32_t)STATUS_BAD_DOF);
        }
      }
    }
    // FP64 geometry once per cell, rounded once to the arithmetic type
    T g[3][3];
    {
      double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, adet = 0.0;
      bool ok = true;
      if (valid) ok = cell_geometry_mode(a.geom, d, a.coords + cell * (d + 1) * d, G, adet);
      if (valid && !ok && kb == 0) atomicOr(a.status, (int32_t)STATUS_DEGENERATE);
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          double v = STIFF ? G[s][t] : ((s == 0 && t == 0) ? adet : 0.0);
          if (!valid) v = 0.0;
          else if (!ok) v = NAN;
          g[s][t] = (T)v;
        }
    }

    ACC acc0[MT], acc1[GZ ? MT : 1];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      acc0[mt] = ACC{0, 0, 0, 0};
      if constexpr (GZ) acc1[mt] = ACC{0, 0, 0, 0};
    }
    if constexpr (STAGE) {
      const V16 *src = (const V16 *)gch;
      V16 *dst = (V16 *)lbuf;
      for (int e = tid; e < nvec; e += NW * 64) dst[e] = src[e];
      __syncthreads();
    }

    for (int qt = 0; qt < a.nqt; ++qt) {
      const T *cur = STAGE ? lbuf + (size_t)(qt & 1) * chunk : gch + (size_t)qt * chunk;
      // the next tile's tables, loaded now and stored to LDS after the math
      V16 pre[STAGE ? PMAX : 1];
      if constexpr (STAGE) {
        if (qt + 1 < a.nqt) {
          const V16 *src = (const V16 *)(gch + (size_t)(qt + 1) * chunk);
#pragma unroll
          for (int p = 0; p < PMAX; ++p) {
            const int e = tid + p * NW * 64;
            if (e < nvec) pre[p] = src[e];
          }
        }
      }

      // evaluation at the 16 points of the tile
      ACC e0[NE], e1[GZ ? NE : 1], ez = ACC{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < NE; ++t) {
        e0[t] = ACC{0, 0, 0, 0};
        if constexpr (GZ) e1[t] = ACC{0, 0, 0, 0};
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const T aop = cur[((STIFF ? 1 + t : 0) * KS + ks) * 64 + lane];
          e0[t] = P::mma(aop, X0[ks], e0[t]);
          if constexpr (GZ) e1[t] = P::mma(aop, X1[ks], e1[t]);
        }
        if constexpr (COEFF) ez = P::mma(cur[ks * 64 + lane], Zk[ks], ez);
      }

      // step 2 and the adjoint density, per point held by this lane
      T rs[NE][4], gq[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T w = cur[W_OFF + P::row(kb, r)];
        const T wz = COEFF ? w * ez[r] : w;
        if constexpr (STIFF) {
          T Gx[3];
#pragma unroll
          for (int s = 0; s < 3; ++s)
            Gx[s] = g[s][0] * e0[0][r] + g[s][1] * e0[1][r] + g[s][2] * e0[2][r];
#pragma unroll
          for (int s = 0; s < 3; ++s) rs[s][r] = wz * Gx[s];
          if constexpr (GZ) gq[r] = w * (e1[0][r] * Gx[0] + e1[1][r] * Gx[1] + e1[2][r] * Gx[2]);
        } else {
          const T gx = g[0][0] * e0[0][r];
          rs[0][r] = wz * gx;
          if constexpr (GZ) gq[r] = w * (e1[0][r] * gx);
        }
      }

      // step 3: v += sum_s B_s r_s (and g += B_0 gq), K = the lane's points
#pragma unroll
      for (int s = 0; s < NE; ++s) {
        const int tab = STIFF ? 1 + s : 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc0[mt] = P::mma(cur[C_OFF + ((tab * MT + mt) * 4 + r) * 64 + lane], rs[s][r],
                              acc0[mt]);
      }
      if constexpr (GZ) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc1[mt] = P::mma(cur[C_OFF + (mt * 4 + r) * 64 + lane], gq[r], acc1[mt]);
      }

      if constexpr (STAGE) {
        if (qt + 1 < a.nqt) {
          V16 *dst = (V16 *)(lbuf + (size_t)((qt + 1) & 1) * chunk);
#pragma unroll
          for (int p = 0; p < PMAX; ++p) {
            const int e = tid + p * NW * 64;
            if (e < nvec) dst[e] = pre[p];
          }
        }
        __syncthreads();
      }
    }

    if (valid) {
      T *o0 = (T *)a.out0 + cell * n_phi;
      T *o1 = GZ ? (T *)a.out1 + cell * n_phi : nullptr;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * mt + P::row(kb, r);
            if (i < n_phi) {
              o0[i] = acc0[mt][r];
              if constexpr (GZ) o1[i] = acc1[mt][r];
            }
          }
    }
  }
}

template <class P, int KS, bool STIFF, bool COEFF, bool GZ>
static fe_status launch_action_one(const ActArgs &k, hipStream_t s) {
  typedef typename P::real T;
  constexpr int NT = STIFF ? 4 : 1, MT = (KS + 3) / 4;
  if (k.nks != KS || k.mt != MT || k.nt != NT ||
      k.chunk != (size_t)64 * (NT * KS + NT * MT * 4 + 1))
    return FE_EINVAL;
  // FP32: tables staged in LDS, 8 waves; FP64: tables read from L2, 4 waves
  // (one per SIMD: the dofs and accumulators of a lane need the registers)
  constexpr bool STAGE = sizeof(T) == 4;
  constexpr int NW = STAGE ? 8 : 4;
  auto kern = action_kernel<P, KS, STIFF, COEFF, GZ, STAGE, NW>;
  const size_t smem = STAGE ? 2 * k.chunk * sizeof(T) : 0;
  if (smem > 160 * 1024) return FE_EUNSUPPORTED;
  LaunchInfo li;
  if (launch_info((const void *)kern, NW * 64, smem, &li) != FE_OK) return FE_EHIP;
  const int ncu = li.ncu, per_cu = li.per_cu;
  if (per_cu < 1) return FE_EUNSUPPORTED;
  const int64_t groups = ((k.n_cells + 15) / 16 + NW - 1) / NW;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(groups, (int64_t)ncu * per_cu));
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), smem, s, k);
  return hipGetLastError() == hipSuccess ? FE_OK : FE_EHIP;
}

template <class P, int KS>
static fe_status launch_action_ks(const ActArgs &k, bool stiff, bool coeff, bool gz,
                                  hipStream_t s) {
  if (stiff) {
    if (gz) return launch_action_one<P, KS, true, true, true>(k, s);
    if (coeff) return launch_action_one<P, KS, true, true, false>(k, s);
    return launch_action_one<P, KS, true, false, false>(k, s);
  }
  if (gz) return launch_action_one<P, KS, false, true, true>(k, s);
  if (coeff) return launch_action_one<P, KS, false, true, false>(k, s);
  return launch_action_one<P, KS, false, false, false>(k, s);
}

template <class P>
fe_status launch_action_impl(const ActionLaunch &a) {
  const FormLayout &L = *a.L;
  if (L.act_nt == 0) return FE_EUNSUPPORTED;
  ActArgs k;
  k.chunks = a.form_buf + L.off_act;
  k.coords = a.coords;
  k.dofmap = a.dofmap;
  k.coeff = a.coeff;
  k.x0 = a.x0;
  k.x1 = a.x1;
  k.out0 = a.out0;
  k.out1 = a.out1;
  k.status = a.status;
  k.n_cells = a.n_cells;
  k.n_dofs = a.n_dofs;
  k.d = L.d;
  k.n_phi = L.n_phi;
  k.nks = L.act_nks;
  k.mt = L.act_mt;
  k.nqt = L.act_nqt;
  k.nt = L.act_nt;
  k.chunk = L.act_chunk;
  k.geom = a.geom;
  const bool stiff = L.form == FE_STIFFNESS, coeff = a.coeff != nullptr,
             gz = a.x1 != nullptr && a.out1 != nullptr;
  if (gz && !coeff) return FE_EINVAL;
  hipStream_t s = (hipStream_t)a.stream;
  switch (k.nks) {
    case 1: return launch_action_ks<P, 1>(k, stiff, coeff, gz, s);
    case 3: return launch_action_ks<P, 3>(k, stiff, coeff, gz, s);
    case 5: return launch_action_ks<P, 5>(k, stiff, coeff, gz, s);
    case 9: return launch_action_ks<P, 9>(k, stiff, coeff, gz, s);
    case 14: return launch_action_ks<P, 14>(k, stiff, coeff, gz, s);
    case 21: return launch_action_ks<P, 21>(k, stiff, coeff, gz, s);
  }
  return FE_EUNSUPPORTED;
}

}  // namespace fe
