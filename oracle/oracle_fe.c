/*
 * Oracle for finite element cell kernels and global assembly, plain FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * library shares no code with it.
 *
 * What it computes (Croci & Wells, "Mixed-precision finite element kernels
 * and assembly"):
 *   - Geometry (Section 4.2): the Jacobian of the affine map from the P1
 *     reference basis (eq. Jacobian_def), det J by LU factorisation with
 *     partial pivoting (the algorithm of the Theorem on LU determinants),
 *     J^{-1} by LU solves, and the geometry tensor
 *         G = |det J|                         (mass form)
 *         G_ij = |det J| sum_k Jinv_ik Jinv_jk (Poisson form).
 *   - Local matrices by Algorithm 1 (Section 3.2): C_st = diag_q(w_q z_q G_st),
 *     H_st = C_st B_t^T, A = sum_s sum_t B_s H_st, where z_q is the
 *     coefficient evaluated at the quadrature points, z_q = sum_k z_k phi_k(X_q)
 *     (Lemma on FE function evaluation), or 1 when there is no coefficient.
 *   - Global assembly A^g = L D L^T (Section 3.3): the sparsity pattern is the
 *     set of all (dof(K,i), dof(K,j)) pairs, rows in dof order, columns
 *     ascending and unique, explicit zeros kept; values summed in FP64 in the
 *     order cell K ascending, then i, then j.
 *
 *   - Local vectors by Algorithm 2 (Section 3.2, linear forms / actions):
 *     the known function w is evaluated at the quadrature points as an FE
 *     function (w_q = sum_k w_k phi_k(X_q), or its reference gradient), then
 *     r_s = vstack_q(w_q z_q (G w_q))  (Poisson; w_q |det J| z_q w_q for mass)
 *     and v = sum_s B_s r_s.
 *   - The coefficient adjoint of f(z) = v^T A(z) u: f is linear in the nodal
 *     values z, z_q = sum_k z_k phi_k(X_q), so on cell K
 *         df/dz_k = sum_q phi_k(X_q) w_q g_q,
 *         g_q = (grad u_h)^T G (grad v_h)   (Poisson),
 *         g_q = |det J| u_h v_h              (mass),
 *     with u_h, v_h evaluated at X_q as FE functions.
 *   - Vector assembly v^g = L b (Section 3.3): local vectors summed into the
 *     global vector in the order cell K ascending, then i.
 *
 *   - Hexahedra (boxed cells): the same Algorithm 1 with the geometry tensor
 *     evaluated at every quadrature point of the trilinear map
 *     (oracle_hex_local_matrices).
 *
 * Tabulations (weights, basis values and gradients at the quadrature points)
 * are inputs; the oracle's own Python side computes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_EDEGENERATE (-5)
#define ORACLE_ENOMEM (-6)

#define FORM_MASS 0
#define FORM_STIFFNESS 1

/* J_ij = sum_k x_i^k d_j phi_k for the P1 reference basis
 * phi_0 = 1 - sum X, phi_k = X_k (k = 1..d); x is [d+1][d]. */
static void jacobian(int d, const double *x, double *J) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = 0.0;
      for (int k = 0; k <= d; ++k) {
        double dphi = (k == 0) ? -1.0 : (k - 1 == j ? 1.0 : 0.0);
        s += x[k * d + i] * dphi;
      }
      J[i * d + j] = s;
    }
}

/* In-place LU with partial pivoting: PA = LU, unit lower L. Returns the
 * permutation sign (+1/-1) or 0 when a zero pivot is met. */
static int lu_factor(int d, double *LU, int *piv) {
  int sign = 1;
  for (int i = 0; i < d; ++i) piv[i] = i;
  for (int k = 0; k < d; ++k) {
    int p = k;
    double best = fabs(LU[k * d + k]);
    for (int r = k + 1; r < d; ++r)
      if (fabs(LU[r * d + k]) > best) { best = fabs(LU[r * d + k]); p = r; }
    if (best == 0.0) return 0;
    if (p != k) {
      for (int c = 0; c < d; ++c) {
        double t = LU[k * d + c]; LU[k * d + c] = LU[p * d + c]; LU[p * d + c] = t;
      }
      int t = piv[k]; piv[k] = piv[p]; piv[p] = t;
      sign = -sign;
    }
    for (int r = k + 1; r < d; ++r) {
      double l = LU[r * d + k] / LU[k * d + k];
      LU[r * d + k] = l;
      for (int c = k + 1; c < d; ++c) LU[r * d + c] -= l * LU[k * d + c];
    }
  }
  return sign;
}

/* Solve A x = b given the LU factors of PA. */
static void lu_solve(int d, const double *LU, const int *piv, const double *b, double *x) {
  double y[3];
  for (int i = 0; i < d; ++i) {
    double s = b[piv[i]];
    for (int k = 0; k < i; ++k) s -= LU[i * d + k] * y[k];
    y[i] = s;
  }
  for (int i = d - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < d; ++k) s -= LU[i * d + k] * x[k];
    x[i] = s / LU[i * d + i];
  }
}

/* Geometry of one affine simplex.  Outputs may be NULL.
 * G_stiff = |det J| J^{-1} J^{-T}; mass geometry is |det J|. */
int oracle_geometry(int d, const double *x, double *J_out, double *det_out,
                    double *Jinv_out, double *G_out) {
  if (d < 2 || d > 3 || !x) return ORACLE_EINVAL;
  double J[9], LU[9], Jinv[9];
  int piv[3];
  jacobian(d, x, J);
  memcpy(LU, J, sizeof(double) * d * d);
  int sign = lu_factor(d, LU, piv);
  double det = 0.0;
  if (sign != 0) {
    det = (double)sign;
    for (int i = 0; i < d; ++i) det *= LU[i * d + i];
  }
  if (J_out) memcpy(J_out, J, sizeof(double) * d * d);
  if (det_out) *det_out = det;
  if (sign == 0 || det == 0.0 || !isfinite(det)) return ORACLE_EDEGENERATE;
  for (int c = 0; c < d; ++c) {
    double e[3] = {0, 0, 0}, col[3];
    e[c] = 1.0;
    lu_solve(d, LU, piv, e, col);
    for (int r = 0; r < d; ++r) Jinv[r * d + c] = col[r];
  }
  if (Jinv_out) memcpy(Jinv_out, Jinv, sizeof(double) * d * d);
  if (G_out) {
    double ad = fabs(det);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += Jinv[i * d + k] * Jinv[j * d + k];
        G_out[i * d + j] = ad * s;
      }
  }
  for (int i = 0; i < d * d; ++i)
    if (!isfinite(Jinv[i])) return ORACLE_EDEGENERATE;
  return ORACLE_OK;
}

/* Local element matrices by Algorithm 1 for every cell.
 *   coords  [n_cells][d+1][d]
 *   weights [n_q]
 *   bval    [n_q][n_phi]      basis values at the quadrature points
 *   bgrad   [d][n_q][n_phi]   reference gradients (stiffness only)
 *   dofmap  [n_cells][n_phi]  (used only with a coefficient)
 *   coeff   [n_dofs] or NULL  nodal coefficient values z
 *   A_out   [n_cells][n_phi][n_phi], row index = first basis index
 * Returns ORACLE_OK or the first error met (ORACLE_EDEGENERATE). */
int oracle_local_matrices(int d, int form, int64_t n_cells, const double *coords,
                          int n_phi, int n_q, const double *weights,
                          const double *bval, const double *bgrad,
                          const int32_t *dofmap, const double *coeff,
                          double *A_out, int nthreads) {
  if (d < 2 || d > 3 || n_phi < 1 || n_q < 1 || !coords || !weights || !A_out)
    return ORACLE_EINVAL;
  if (form != FORM_MASS && form != FORM_STIFFNESS) return ORACLE_EINVAL;
  if (form == FORM_STIFFNESS && !bgrad) return ORACLE_EINVAL;
  if (!bval) return ORACLE_EINVAL;
  if (coeff && !dofmap) return ORACLE_EINVAL;
  const int nd = (form == FORM_MASS) ? 1 : d;
  int status = ORACLE_OK;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    /* B_s^T laid out [s][i][q] so the q-sums read contiguously. */
    double *BT = (double *)malloc(sizeof(double) * nd * n_phi * n_q);
    double *HT = (double *)malloc(sizeof(double) * nd * nd * n_phi * n_q);
    double *z = (double *)malloc(sizeof(double) * n_q);
    if (!BT || !HT || !z) {
#pragma omp atomic write
      status = ORACLE_ENOMEM;
    } else {
      /* Step 1 (tabulation) is an input: copy it into [s][i][q]. */
      for (int s = 0; s < nd; ++s)
        for (int i = 0; i < n_phi; ++i)
          for (int q = 0; q < n_q; ++q)
            BT[((size_t)s * n_phi + i) * n_q + q] =
                (form == FORM_MASS) ? bval[(size_t)q * n_phi + i]
                                    : bgrad[((size_t)s * n_q + q) * n_phi + i];
#pragma omp for schedule(static)
      for (int64_t K = 0; K < n_cells; ++K) {
        double G[9], det;
        int st = oracle_geometry(d, coords + K * (d + 1) * d, NULL, &det, NULL, G);
        double *A = A_out + (size_t)K * n_phi * n_phi;
        if (st != ORACLE_OK) {
#pragma omp atomic write
          status = st;
          for (int e = 0; e < n_phi * n_phi; ++e) A[e] = NAN;
          continue;
        }
        if (form == FORM_MASS) G[0] = fabs(det);
        /* coefficient at the quadrature points */
        for (int q = 0; q < n_q; ++q) {
          double zq = 1.0;
          if (coeff) {
            zq = 0.0;
            for (int k = 0; k < n_phi; ++k)
              zq += coeff[dofmap[(size_t)K * n_phi + k]] * bval[(size_t)q * n_phi + k];
          }
          z[q] = zq;
        }
        /* Steps 2-3: C_st[q] = w_q z_q G_st and H_st = C_st B_t^T, stored as
         * H_st^T [s][t][j][q]. */
        for (int s = 0; s < nd; ++s)
          for (int t = 0; t < nd; ++t) {
            double g = G[s * nd + t];
            for (int j = 0; j < n_phi; ++j) {
              const double *bt = BT + ((size_t)t * n_phi + j) * n_q;
              double *h = HT + (((size_t)s * nd + t) * n_phi + j) * n_q;
              for (int q = 0; q < n_q; ++q) h[q] = (weights[q] * z[q] * g) * bt[q];
            }
          }
        /* Step 4: A = sum_s sum_t B_s H_st. */
        for (int i = 0; i < n_phi; ++i)
          for (int j = 0; j < n_phi; ++j) {
            double acc = 0.0;
            for (int s = 0; s < nd; ++s) {
              const double *bs = BT + ((size_t)s * n_phi + i) * n_q;
              for (int t = 0; t < nd; ++t) {
                const double *h = HT + (((size_t)s * nd + t) * n_phi + j) * n_q;
                for (int q = 0; q < n_q; ++q) acc += bs[q] * h[q];
              }
            }
            A[(size_t)i * n_phi + j] = acc;
          }
      }
    }
    free(BT); free(HT); free(z);
  }
  return status;
}

/* Hexahedra (boxed cells, Section 5.1 reference cube [0,1]^3): the
 * trilinear map x(X) = sum_v x_v phi_v(X) over the 8 vertices, vertex v at
 * the reference corner (v & 1, (v >> 1) & 1, (v >> 2) & 1), so
 *     J_ij(X) = sum_v x_v,i d_j phi_v(X),
 * which varies over the cell (Section 4.2: the geometry tensor is evaluated
 * at every quadrature point).  X is [3], x8 is [8][3]. */
static void hex_jacobian(const double *x8, const double *X, double *J) {
  for (int e = 0; e < 9; ++e) J[e] = 0.0;
  for (int v = 0; v < 8; ++v) {
    double f[3], df[3];
    for (int e = 0; e < 3; ++e) {
      int b = (v >> e) & 1;
      f[e] = b ? X[e] : 1.0 - X[e];
      df[e] = b ? 1.0 : -1.0;
    }
    double g[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) J[i * 3 + j] += x8[v * 3 + i] * g[j];
  }
}

/* Geometry tensor of a hexahedron at one point: |det J| (mass) or
 * |det J| J^{-1} J^{-T} (Poisson), det J by LU with partial pivoting and
 * J^{-1} by LU solves, as for simplices. */
static int hex_point_geometry(const double *x8, const double *X, int form, double *G) {
  double J[9], LU[9], Jinv[9];
  int piv[3];
  hex_jacobian(x8, X, J);
  memcpy(LU, J, sizeof J);
  int sign = lu_factor(3, LU, piv);
  if (sign == 0) return ORACLE_EDEGENERATE;
  double det = (double)sign * LU[0] * LU[4] * LU[8];
  if (det == 0.0 || !isfinite(det)) return ORACLE_EDEGENERATE;
  if (form == FORM_MASS) {
    G[0] = fabs(det);
    return ORACLE_OK;
  }
  for (int c = 0; c < 3; ++c) {
    double e[3] = {0, 0, 0}, col[3];
    e[c] = 1.0;
    lu_solve(3, LU, piv, e, col);
    for (int r = 0; r < 3; ++r) Jinv[r * 3 + c] = col[r];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Jinv[i * 3 + k] * Jinv[j * 3 + k];
      G[i * 3 + j] = fabs(det) * s;
      if (!isfinite(G[i * 3 + j])) return ORACLE_EDEGENERATE;
    }
  return ORACLE_OK;
}

/* Local element matrices of trilinear hexahedra by Algorithm 1 with a
 * geometry tensor per quadrature point:
 *   C_st = diag_q(w_q G_st(X_q)), H_st = C_st B_t^T, A = sum_s sum_t B_s H_st.
 *   coords  [n_cells][8][3]
 *   points  [n_q][3], weights [n_q]
 *   bval    [n_q][n_phi], bgrad [3][n_q][n_phi] (stiffness only)
 *   A_out   [n_cells][n_phi][n_phi]
 * Returns ORACLE_OK or the first error met (ORACLE_EDEGENERATE: det J = 0 or
 * not finite at some point; that cell's matrix is NaN). */
int oracle_hex_local_matrices(int form, int64_t n_cells, const double *coords, int n_phi,
                              int n_q, const double *points, const double *weights,
                              const double *bval, const double *bgrad, double *A_out,
                              int nthreads) {
  if (n_phi < 1 || n_q < 1 || !coords || !points || !weights || !bval || !A_out)
    return ORACLE_EINVAL;
  if (form != FORM_MASS && form != FORM_STIFFNESS) return ORACLE_EINVAL;
  if (form == FORM_STIFFNESS && !bgrad) return ORACLE_EINVAL;
  const int nd = (form == FORM_MASS) ? 1 : 3;
  int status = ORACLE_OK;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    double *BT = (double *)malloc(sizeof(double) * nd * n_phi * n_q);
    double *HT = (double *)malloc(sizeof(double) * nd * nd * n_phi * n_q);
    double *C = (double *)malloc(sizeof(double) * nd * nd * n_q);
    if (!BT || !HT || !C) {
#pragma omp atomic write
      status = ORACLE_ENOMEM;
    } else {
      for (int s = 0; s < nd; ++s)
        for (int i = 0; i < n_phi; ++i)
          for (int q = 0; q < n_q; ++q)
            BT[((size_t)s * n_phi + i) * n_q + q] =
                (form == FORM_MASS) ? bval[(size_t)q * n_phi + i]
                                    : bgrad[((size_t)s * n_q + q) * n_phi + i];
#pragma omp for schedule(static)
      for (int64_t K = 0; K < n_cells; ++K) {
        double *A = A_out + (size_t)K * n_phi * n_phi;
        int st = ORACLE_OK;
        /* Step 2: C_st(q) = w_q G_st(X_q) */
        for (int q = 0; q < n_q && st == ORACLE_OK; ++q) {
          double G[9];
          st = hex_point_geometry(coords + K * 24, points + 3 * q, form, G);
          for (int s = 0; s < nd; ++s)
            for (int t = 0; t < nd; ++t) C[((size_t)s * nd + t) * n_q + q] = weights[q] * G[s * nd + t];
        }
        if (st != ORACLE_OK) {
#pragma omp atomic write
          status = st;
          for (int e = 0; e < n_phi * n_phi; ++e) A[e] = NAN;
          continue;
        }
        /* Step 3: H_st = C_st B_t^T, stored as H_st^T [s][t][j][q] */
        for (int s = 0; s < nd; ++s)
          for (int t = 0; t < nd; ++t) {
            const double *c = C + ((size_t)s * nd + t) * n_q;
            for (int j = 0; j < n_phi; ++j) {
              const double *bt = BT + ((size_t)t * n_phi + j) * n_q;
              double *h = HT + (((size_t)s * nd + t) * n_phi + j) * n_q;
              for (int q = 0; q < n_q; ++q) h[q] = c[q] * bt[q];
            }
          }
        /* Step 4: A = sum_s sum_t B_s H_st */
        for (int i = 0; i < n_phi; ++i)
          for (int j = 0; j < n_phi; ++j) {
            double acc = 0.0;
            for (int s = 0; s < nd; ++s) {
              const double *bs = BT + ((size_t)s * n_phi + i) * n_q;
              for (int t = 0; t < nd; ++t) {
                const double *h = HT + (((size_t)s * nd + t) * n_phi + j) * n_q;
                for (int q = 0; q < n_q; ++q) acc += bs[q] * h[q];
              }
            }
            A[(size_t)i * n_phi + j] = acc;
          }
      }
    }
    free(BT); free(HT); free(C);
  }
  return status;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Sparsity pattern of A^g = L D L^T.  With col_idx == NULL only row_ptr
 * [n_dofs+1] is filled; the return value is nnz (or a negative error). */
int64_t oracle_csr_pattern(int64_t n_cells, int n_phi, const int32_t *dofmap,
                           int64_t n_dofs, int64_t *row_ptr, int32_t *col_idx) {
  if (n_cells < 0 || n_phi < 1 || n_dofs < 1 || !dofmap || !row_ptr) return ORACLE_EINVAL;
  for (int64_t e = 0; e < n_cells * n_phi; ++e)
    if (dofmap[e] < 0 || dofmap[e] >= n_dofs) return ORACLE_EINVAL;
  /* dof -> incident cells */
  int64_t *cnt = (int64_t *)calloc((size_t)n_dofs + 1, sizeof(int64_t));
  if (!cnt) return ORACLE_ENOMEM;
  for (int64_t e = 0; e < n_cells * n_phi; ++e) cnt[dofmap[e] + 1]++;
  for (int64_t g = 0; g < n_dofs; ++g) cnt[g + 1] += cnt[g];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_dofs);
  int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_cells * n_phi + 1));
  if (!fill || !adj) { free(cnt); free(fill); free(adj); return ORACLE_ENOMEM; }
  memcpy(fill, cnt, sizeof(int64_t) * (size_t)n_dofs);
  for (int64_t K = 0; K < n_cells; ++K)
    for (int i = 0; i < n_phi; ++i) adj[fill[dofmap[K * n_phi + i]]++] = K;
  int64_t cap = 64;
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * cap);
  int64_t nnz = 0;
  row_ptr[0] = 0;
  for (int64_t g = 0; g < n_dofs; ++g) {
    int64_t m = (cnt[g + 1] - cnt[g]) * n_phi;
    if (m > cap) {
      cap = m;
      buf = (int32_t *)realloc(buf, sizeof(int32_t) * cap);
    }
    int64_t k = 0;
    for (int64_t a = cnt[g]; a < cnt[g + 1]; ++a)
      for (int j = 0; j < n_phi; ++j) buf[k++] = dofmap[adj[a] * n_phi + j];
    qsort(buf, (size_t)k, sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t a = 0; a < k; ++a)
      if (a == 0 || buf[a] != buf[a - 1]) buf[u++] = buf[a];
    if (col_idx) memcpy(col_idx + nnz, buf, sizeof(int32_t) * (size_t)u);
    nnz += u;
    row_ptr[g + 1] = nnz;
  }
  free(buf); free(cnt); free(fill); free(adj);
  return nnz;
}

/* values = L D L^T on a given pattern, summed in the order K, i, j. */
int oracle_assemble(int64_t n_cells, int n_phi, const int32_t *dofmap,
                    const double *A_local, int64_t n_dofs, const int64_t *row_ptr,
                    const int32_t *col_idx, double *values) {
  if (!dofmap || !A_local || !row_ptr || !col_idx || !values) return ORACLE_EINVAL;
  memset(values, 0, sizeof(double) * (size_t)row_ptr[n_dofs]);
  for (int64_t K = 0; K < n_cells; ++K)
    for (int i = 0; i < n_phi; ++i) {
      int32_t g = dofmap[K * n_phi + i];
      const int32_t *cols = col_idx + row_ptr[g];
      int64_t len = row_ptr[g + 1] - row_ptr[g];
      for (int j = 0; j < n_phi; ++j) {
        int32_t h = dofmap[K * n_phi + j];
        int64_t lo = 0, hi = len - 1, pos = -1;
        while (lo <= hi) {
          int64_t mid = (lo + hi) / 2;
          if (cols[mid] == h) { pos = mid; break; }
          if (cols[mid] < h) lo = mid + 1; else hi = mid - 1;
        }
        if (pos < 0) return ORACLE_EINVAL;
        values[row_ptr[g] + pos] += A_local[((size_t)K * n_phi + i) * n_phi + j];
      }
    }
  return ORACLE_OK;
}

/* FE function evaluation on cell K at every quadrature point:
 *   val[q]      = sum_k x_{L(K,k)} phi_k(X_q)
 *   grad[t][q]  = sum_k x_{L(K,k)} d_t phi_k(X_q)   (when grad and bgrad are given)
 * (the Lemma on FE function evaluation). */
static void fe_eval(int d, int64_t K, int n_phi, int n_q, const double *bval,
                    const double *bgrad, const int32_t *dofmap, const double *x,
                    double *val, double *grad) {
  for (int q = 0; q < n_q; ++q) {
    double a = 0.0;
    for (int k = 0; k < n_phi; ++k) a += x[dofmap[K * n_phi + k]] * bval[(size_t)q * n_phi + k];
    val[q] = a;
    if (grad && bgrad)
      for (int t = 0; t < d; ++t) {
        double b = 0.0;
        for (int k = 0; k < n_phi; ++k)
          b += x[dofmap[K * n_phi + k]] * bgrad[((size_t)t * n_q + q) * n_phi + k];
        grad[(size_t)t * n_q + q] = b;
      }
  }
}

/* Local vectors of every cell by Algorithm 2 (v_out [n_cells][n_phi]) for the
 * action of the mass or Poisson form with coefficient z (NULL: z = 1) on the
 * global FE function u, and, when g_out != NULL, the local coefficient
 * adjoint g_out [n_cells][n_phi] of f(z) = vv^T A(z) u (vv must then be given).
 * Either output may be NULL. */
int oracle_local_vectors(int d, int form, int64_t n_cells, const double *coords, int n_phi,
                         int n_q, const double *weights, const double *bval,
                         const double *bgrad, const int32_t *dofmap, const double *coeff,
                         const double *u, const double *vv, double *v_out, double *g_out,
                         int nthreads) {
  if (d < 2 || d > 3 || n_phi < 1 || n_q < 1 || !coords || !weights || !bval || !dofmap || !u)
    return ORACLE_EINVAL;
  if (form != FORM_MASS && form != FORM_STIFFNESS) return ORACLE_EINVAL;
  if (form == FORM_STIFFNESS && !bgrad) return ORACLE_EINVAL;
  if (g_out && !vv) return ORACLE_EINVAL;
  const int nd = (form == FORM_MASS) ? 1 : d;
  int status = ORACLE_OK;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    double *uq = (double *)malloc(sizeof(double) * n_q * (1 + d));
    double *vq = (double *)malloc(sizeof(double) * n_q * (1 + d));
    double *zq = (double *)malloc(sizeof(double) * n_q);
    double *r = (double *)malloc(sizeof(double) * n_q * nd);
    if (!uq || !vq || !zq || !r) {
#pragma omp atomic write
      status = ORACLE_ENOMEM;
    } else {
#pragma omp for schedule(static)
      for (int64_t K = 0; K < n_cells; ++K) {
        double G[9], det;
        int st = oracle_geometry(d, coords + K * (d + 1) * d, NULL, &det, NULL, G);
        if (st != ORACLE_OK) {
#pragma omp atomic write
          status = st;
          for (int i = 0; i < n_phi; ++i) {
            if (v_out) v_out[K * n_phi + i] = NAN;
            if (g_out) g_out[K * n_phi + i] = NAN;
          }
          continue;
        }
        if (form == FORM_MASS) G[0] = fabs(det);
        /* coefficient and the known functions at the quadrature points */
        for (int q = 0; q < n_q; ++q) zq[q] = 1.0;
        if (coeff) fe_eval(d, K, n_phi, n_q, bval, NULL, dofmap, coeff, zq, NULL);
        fe_eval(d, K, n_phi, n_q, bval, form == FORM_STIFFNESS ? bgrad : NULL, dofmap, u, uq,
                uq + n_q);
        if (v_out) {
          /* step 2: r_s(q) = w_q z_q (G grad u)_s, or w_q z_q |det J| u_q */
          for (int s = 0; s < nd; ++s)
            for (int q = 0; q < n_q; ++q) {
              double a = 0.0;
              if (form == FORM_MASS) a = G[0] * uq[q];
              else
                for (int t = 0; t < d; ++t) a += G[s * d + t] * uq[(size_t)(1 + t) * n_q + q];
              r[(size_t)s * n_q + q] = weights[q] * zq[q] * a;
            }
          /* step 3: v = sum_s B_s r_s, B_s[i][q] = d_s phi_i(X_q) (phi_i for mass) */
          for (int i = 0; i < n_phi; ++i) {
            double a = 0.0;
            for (int s = 0; s < nd; ++s)
              for (int q = 0; q < n_q; ++q) {
                const double b = (form == FORM_MASS) ? bval[(size_t)q * n_phi + i]
                                                     : bgrad[((size_t)s * n_q + q) * n_phi + i];
                a += b * r[(size_t)s * n_q + q];
              }
            v_out[K * n_phi + i] = a;
          }
        }
        if (g_out) {
          fe_eval(d, K, n_phi, n_q, bval, form == FORM_STIFFNESS ? bgrad : NULL, dofmap, vv, vq,
                  vq + n_q);
          for (int i = 0; i < n_phi; ++i) {
            double a = 0.0;
            for (int q = 0; q < n_q; ++q) {
              double gq = 0.0;
              if (form == FORM_MASS) gq = G[0] * uq[q] * vq[q];
              else
                for (int s = 0; s < d; ++s)
                  for (int t = 0; t < d; ++t)
                    gq += vq[(size_t)(1 + s) * n_q + q] * G[s * d + t] * uq[(size_t)(1 + t) * n_q + q];
              a += bval[(size_t)q * n_phi + i] * weights[q] * gq;
            }
            g_out[K * n_phi + i] = a;
          }
        }
      }
    }
    free(uq); free(vq); free(zq); free(r);
  }
  return status;
}

/* v^g = L b: local vectors b [n_cells][n_phi] summed into out [n_dofs] in the
 * order cell K ascending, then i. */
int oracle_assemble_vector(int64_t n_cells, int n_phi, const int32_t *dofmap, const double *b,
                           int64_t n_dofs, double *out) {
  if (!dofmap || !b || !out || n_dofs < 1) return ORACLE_EINVAL;
  memset(out, 0, sizeof(double) * (size_t)n_dofs);
  for (int64_t K = 0; K < n_cells; ++K)
    for (int i = 0; i < n_phi; ++i) {
      const int32_t g = dofmap[K * n_phi + i];
      if (g < 0 || g >= n_dofs) return ORACLE_EINVAL;
      out[g] += b[K * n_phi + i];
    }
  return ORACLE_OK;
}
