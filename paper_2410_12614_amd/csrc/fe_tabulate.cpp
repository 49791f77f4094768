// Host-side reference tabulation (FP64): collapsed Gauss-Jacobi quadrature
// and the product-form Lagrange basis with its gradients.
//
// Algorithm 1 step 1 (Section 3.2); tables B of Section 3.1; product-form
// basis and product-rule derivatives of Appendix A.  Quadrature nodes are
// the zeros of Jacobi polynomials P_m^(alpha,0), found by Newton's method with
// deflation on the three-term recurrence; weights from the closed-form
// Christoffel numbers.
#include <cmath>
#include <cstring>
#include <vector>

#include "fe_internal.h"

namespace fe {

namespace {

// P_n^(a,b)(x) and P_{n-1}^(a,b)(x) by the three-term recurrence.
void jacobi_pair(int n, double a, double b, double x, double *pn, double *pnm1) {
  double p0 = 1.0;
  if (n == 0) {
    *pn = p0;
    *pnm1 = 0.0;
    return;
  }
  double p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int k = 1; k < n; ++k) {
    double s = 2.0 * k + a + b;
    double c1 = 2.0 * (k + 1) * (k + a + b + 1.0) * s;
    double c2 = (s + 1.0) * (s * (s + 2.0) * x + a * a - b * b);
    double c3 = 2.0 * (k + a) * (k + b) * (s + 2.0);
    double p2 = (c2 * p1 - c3 * p0) / c1;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *pnm1 = p0;
}

// Derivative from (2n+a+b)(1-x^2) P_n' = n[(a-b) - (2n+a+b) x] P_n + 2(n+a)(n+b) P_{n-1}.
double jacobi_deriv(int n, double a, double b, double x, double pn, double pnm1) {
  double s = 2.0 * n + a + b;
  return (n * ((a - b) - s * x) * pn + 2.0 * (n + a) * (n + b) * pnm1) / (s * (1.0 - x * x));
}

}  // namespace

// m-point Gauss-Jacobi rule on [0,1] for the weight (1-t)^alpha.
void gauss_jacobi_01(int m, int alpha, double *t, double *w) {
  const double a = alpha, b = 0.0;
  std::vector<double> x(m);
  for (int k = 0; k < m; ++k) {
    // initial guess: Chebyshev-like angle, then Newton with deflation of the
    // zeros already found (they are found in descending order)
    double th = M_PI * (k + 0.75 + 0.5 * a) / (m + 0.5 + 0.5 * (a + b));
    double r = std::cos(th);
    for (int it = 0; it < 100; ++it) {
      double pn, pnm1;
      jacobi_pair(m, a, b, r, &pn, &pnm1);
      double dp = jacobi_deriv(m, a, b, r, pn, pnm1);
      double defl = 0.0;
      for (int j = 0; j < k; ++j) defl += 1.0 / (r - x[j]);
      double delta = pn / (dp - defl * pn);
      r -= delta;
      if (std::fabs(delta) <= 1e-16 * std::max(1.0, std::fabs(r))) break;
    }
    x[k] = r;
  }
  // Christoffel numbers on [-1,1]:
  // w = 2^(a+b+1) G(m+a+1) G(m+b+1) / (G(m+a+b+1) m!) / ((1-x^2) P_m'(x)^2)
  double lc = std::lgamma(m + a + 1.0) + std::lgamma(m + b + 1.0) - std::lgamma(m + a + b + 1.0) -
              std::lgamma(m + 1.0);
  double cst = std::exp(lc) * std::pow(2.0, a + b + 1.0);
  for (int k = 0; k < m; ++k) {
    double pn, pnm1;
    jacobi_pair(m, a, b, x[k], &pn, &pnm1);
    double dp = jacobi_deriv(m, a, b, x[k], pn, pnm1);
    double wk = cst / ((1.0 - x[k] * x[k]) * dp * dp);
    // ascending t order
    int o = m - 1 - k;
    t[o] = 0.5 * (x[k] + 1.0);
    w[o] = wk * std::pow(2.0, -(a + b + 1.0));
  }
}

int simplex_dim(int d, int p) {
  int num = 1, den = 1;
  for (int j = 1; j <= d; ++j) {
    num *= p + j;
    den *= j;
  }
  return num / den;
}

// Local multi-indices, alpha_d outermost, alpha_1 innermost: out[n_phi][d].
void lattice_indices(int d, int p, std::vector<int> &out) {
  out.clear();
  if (d == 2) {
    for (int a2 = 0; a2 <= p; ++a2)
      for (int a1 = 0; a1 <= p - a2; ++a1) {
        out.push_back(a1);
        out.push_back(a2);
      }
  } else {
    for (int a3 = 0; a3 <= p; ++a3)
      for (int a2 = 0; a2 <= p - a3; ++a2)
        for (int a1 = 0; a1 <= p - a3 - a2; ++a1) {
          out.push_back(a1);
          out.push_back(a2);
          out.push_back(a3);
        }
  }
}

// phi_alpha(X) = prod_{i=0..d} prod_{j<alpha_i} (p lambda_i - j)/(j+1),
// lambda_0 = 1 - sum X, lambda_i = X_i; gradient by the product rule.
void lagrange_eval(int d, int p, const double *X, double *val, double *grad /*[d][n_phi] or NULL*/) {
  std::vector<int> idx;
  lattice_indices(d, p, idx);
  const int nphi = (int)idx.size() / d;
  double lam[4];
  lam[0] = 1.0;
  for (int i = 0; i < d; ++i) {
    lam[i + 1] = X[i];
    lam[0] -= X[i];
  }
  double fac[32];
  int owner[32];
  for (int a = 0; a < nphi; ++a) {
    int alpha[4];
    alpha[0] = p;
    for (int i = 0; i < d; ++i) {
      alpha[i + 1] = idx[a * d + i];
      alpha[0] -= alpha[i + 1];
    }
    int nf = 0;
    for (int i = 0; i <= d; ++i)
      for (int j = 0; j < alpha[i]; ++j) {
        fac[nf] = (p * lam[i] - j) / (j + 1.0);
        owner[nf] = i;
        ++nf;
      }
    double v = 1.0;
    for (int f = 0; f < nf; ++f) v *= fac[f];
    val[a] = v;
    if (grad) {
      for (int s = 0; s < d; ++s) grad[s * nphi + a] = 0.0;
      for (int f = 0; f < nf; ++f) {
        double others = 1.0;
        for (int g = 0; g < nf; ++g)
          if (g != f) others *= fac[g];
        // d fac_f / d X_s = p * d lambda_i / d X_s / (j+1); recover 1/(j+1) from
        // the factor's own formula: fac = (p lam - j)/(j+1)
        int i = owner[f];
        int j = 0;
        for (int g = 0; g < f; ++g)
          if (owner[g] == i) ++j;
        double scale = p / (j + 1.0);
        for (int s = 0; s < d; ++s) {
          double dl = (i == 0) ? -1.0 : (i - 1 == s ? 1.0 : 0.0);
          grad[s * nphi + a] += scale * dl * others;
        }
      }
    }
  }
}

}  // namespace fe

using namespace fe;

namespace fe {
// Equispaced 1D Lagrange basis of degree p on [0, 1] (nodes k / p) and its
// derivative at t, by the product formula.
static void lagrange_1d(int p, double t, double *v, double *dv) {
  for (int k = 0; k <= p; ++k) {
    double val = 1.0, der = 0.0;
    for (int a = 0; a <= p; ++a) {
      if (a == k) continue;
      const double den = (double)(k - a) / p;
      const double f = (t - (double)a / p) / den;
      der = der * f + val / den;
      val *= f;
    }
    v[k] = val;
    dv[k] = der;
  }
}

// The unit cube [0,1]^3: tensor Gauss-Legendre points (m = floor(q/2)+1 per
// direction, x fastest) and the tensor-product Lagrange basis on the
// equispaced lattice, local index i + (p+1)(j + (p+1)k) for the node
// (i, j, k) / p, with its gradient by the product rule.
static fe_status tabulate_hex(int degree, int quad_degree, int nderiv, int32_t *n_phi,
                              int32_t *n_q, double *points, double *weights, double *table) {
  const int m = quad_degree / 2 + 1, p = degree, n1 = p + 1;
  const int nq = m * m * m, nphi = n1 * n1 * n1;
  *n_phi = nphi;
  *n_q = nq;
  if (!points && !weights && !table) return FE_OK;
  double t[16], w[16];
  gauss_jacobi_01(m, 0, t, w);
  std::vector<double> v1((size_t)m * n1), d1((size_t)m * n1);
  for (int a = 0; a < m; ++a) lagrange_1d(p, t[a], &v1[(size_t)a * n1], &d1[(size_t)a * n1]);
  const size_t slab = (size_t)nq * nphi;
  int q = 0;
  for (int c = 0; c < m; ++c)
    for (int b = 0; b < m; ++b)
      for (int a = 0; a < m; ++a, ++q) {
        if (points) {
          points[q * 3 + 0] = t[a];
          points[q * 3 + 1] = t[b];
          points[q * 3 + 2] = t[c];
        }
        if (weights) weights[q] = w[a] * w[b] * w[c];
        if (!table) continue;
        const double *va = &v1[(size_t)a * n1], *vb = &v1[(size_t)b * n1], *vc = &v1[(size_t)c * n1];
        const double *da = &d1[(size_t)a * n1], *db = &d1[(size_t)b * n1], *dc = &d1[(size_t)c * n1];
        for (int k = 0; k < n1; ++k)
          for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
              const size_t idx = (size_t)q * nphi + i + (size_t)n1 * (j + (size_t)n1 * k);
              table[idx] = va[i] * vb[j] * vc[k];
              if (nderiv) {
                table[slab + idx] = da[i] * vb[j] * vc[k];
                table[2 * slab + idx] = va[i] * db[j] * vc[k];
                table[3 * slab + idx] = va[i] * vb[j] * dc[k];
              }
            }
      }
  return FE_OK;
}
}  // namespace fe

extern "C" fe_status fe_tabulate(int32_t cell, int32_t degree, int32_t quad_degree,
                                 int32_t nderiv, int32_t *n_phi, int32_t *n_q, double *points,
                                 double *weights, double *table) {
  if (cell != FE_TRIANGLE && cell != FE_TETRAHEDRON && cell != FE_HEXAHEDRON) return FE_EINVAL;
  if (degree < 1 || quad_degree < 0 || (nderiv != 0 && nderiv != 1)) return FE_EINVAL;
  if (!n_phi || !n_q) return FE_EINVAL;
  if (degree > FE_MAX_DEGREE || quad_degree > FE_MAX_QUAD_DEGREE) return FE_EUNSUPPORTED;
  if (cell == FE_HEXAHEDRON && degree > FE_MAX_BOX_DEGREE) return FE_EUNSUPPORTED;
  if (cell == FE_HEXAHEDRON)
    return tabulate_hex(degree, quad_degree, nderiv, n_phi, n_q, points, weights, table);
  const int d = cell;
  const int m = quad_degree / 2 + 1;
  const int nq = (d == 2) ? m * m : m * m * m;
  const int nphi = simplex_dim(d, degree);
  *n_phi = nphi;
  *n_q = nq;
  if (!points && !weights && !table) return FE_OK;
  double ta[16], wa[16], tb[16], wb[16], tc[16], wc[16];
  gauss_jacobi_01(m, 0, ta, wa);
  gauss_jacobi_01(m, 1, tb, wb);
  if (d == 3) gauss_jacobi_01(m, 2, tc, wc);
  std::vector<double> X((size_t)nq * d), W(nq);
  int q = 0;
  const int mc = (d == 3) ? m : 1;
  for (int ic = 0; ic < mc; ++ic)
    for (int ib = 0; ib < m; ++ib)
      for (int ia = 0; ia < m; ++ia, ++q) {
        if (d == 2) {
          X[q * 2 + 0] = ta[ia] * (1.0 - tb[ib]);
          X[q * 2 + 1] = tb[ib];
          W[q] = wa[ia] * wb[ib];
        } else {
          X[q * 3 + 0] = ta[ia] * (1.0 - tb[ib]) * (1.0 - tc[ic]);
          X[q * 3 + 1] = tb[ib] * (1.0 - tc[ic]);
          X[q * 3 + 2] = tc[ic];
          W[q] = wa[ia] * wb[ib] * wc[ic];
        }
      }
  if (points) std::memcpy(points, X.data(), sizeof(double) * X.size());
  if (weights) std::memcpy(weights, W.data(), sizeof(double) * W.size());
  if (table) {
    std::vector<double> val(nphi), grad((size_t)d * nphi);
    const size_t slab = (size_t)nq * nphi;
    for (int qq = 0; qq < nq; ++qq) {
      lagrange_eval(d, degree, &X[(size_t)qq * d], val.data(), nderiv ? grad.data() : nullptr);
      std::memcpy(table + (size_t)qq * nphi, val.data(), sizeof(double) * nphi);
      if (nderiv)
        for (int s = 0; s < d; ++s)
          std::memcpy(table + (1 + s) * slab + (size_t)qq * nphi, grad.data() + (size_t)s * nphi,
                      sizeof(double) * nphi);
    }
  }
  return FE_OK;
}

extern "C" const char *fe_status_string(fe_status s) {
  switch (s) {
    case FE_OK: return "success";
    case FE_EINVAL: return "invalid argument";
    case FE_EUNSUPPORTED: return "unsupported cell, degree, quadrature or precision";
    case FE_EOVERFLOW: return "index does not fit its integer type";
    case FE_EHIP: return "HIP runtime error";
    case FE_EDEGENERATE: return "degenerate cell (det J == 0 or non-finite geometry)";
    case FE_ESIZE: return "buffer smaller than the queried size";
    default: return "unknown status";
  }
}

extern "C" const char *fe_version(void) { return "fe-mi355x 0.1"; }
