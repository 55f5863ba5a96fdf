// coeffs.cpp -- host-side collocation coefficients of one HSDC level, FP64
// (computed in long double and rounded):
//   * Radau IIA nodes c_1 < ... < c_M = 1 (Sec. 3.1.2): roots of
//     P_M(2c-1) - P_{M-1}(2c-1), located by a sign scan and refined by bisection;
//   * w_j^k = l_j^{(k)}(0), the weights of Fornberg's finite-difference algorithm
//     (B. Fornberg, Math. Comp. 51, 1988) for derivatives of order 0..M-1 at 0
//     from the values at c_1..c_M (Appendix A, eq. fornberg);
//   * a(0) = Q with q_ij = sum_k c_i^k w_j^{k-1} / k! (eq. def_aij_computable at
//     z = 0, the standard collocation weights);
//   * Lagrange time transfer matrices R and T between two node sets (Sec. 3.2).
#include <cmath>
#include <vector>

#include "hsdc_internal.h"

namespace hsdc {

static long double legendre(int n, long double x) {
  if (n == 0) return 1.0L;
  long double p0 = 1.0L, p1 = x;
  for (int k = 2; k <= n; ++k) {
    const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

static long double radau_poly(int M, long double x) { return legendre(M, x) - legendre(M - 1, x); }

bool radau_nodes(int M, double *c) {
  if (M < 1 || M > MAXM) return false;
  if (M == 1) {
    c[0] = 1.0;
    return true;
  }
  // M-1 interior roots in (-1, 1) plus x = 1
  const int nscan = 200000;
  int found = 0;
  long double xa = -1.0L, fa = radau_poly(M, xa);
  for (int s = 1; s <= nscan && found < M - 1; ++s) {
    const long double xb = -1.0L + 2.0L * s / nscan;
    const long double fb = radau_poly(M, xb);
    if (xb < 1.0L - 1e-12L && ((fa < 0) != (fb < 0))) {
      long double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200; ++it) {
        const long double mid = 0.5L * (lo + hi);
        const long double fm = radau_poly(M, mid);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      c[found++] = (double)(0.5L * (0.5L * (lo + hi) + 1.0L));
    }
    xa = xb;
    fa = fb;
  }
  if (found != M - 1) return false;
  c[M - 1] = 1.0;
  return true;
}

// Fornberg's recursion: weights delta[k][j] such that p^{(k)}(z0) = sum_j delta[k][j] p(x_j)
// for polynomials of degree < n through the n nodes x.
static void fornberg_weights(int n, const long double *x, long double z0, int mmax,
                             std::vector<std::vector<long double>> &delta) {
  delta.assign(mmax + 1, std::vector<long double>(n, 0.0L));
  long double c1 = 1.0L, c4 = x[0] - z0;
  delta[0][0] = 1.0L;
  for (int i = 1; i < n; ++i) {
    const int mn = i < mmax ? i : mmax;
    long double c2 = 1.0L;
    const long double c5 = c4;
    c4 = x[i] - z0;
    for (int j = 0; j < i; ++j) {
      const long double c3 = x[i] - x[j];
      c2 *= c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k)
          delta[k][i] = c1 * (k * delta[k - 1][i - 1] - c5 * delta[k][i - 1]) / c2;
        delta[0][i] = -c1 * c5 * delta[0][i - 1] / c2;
      }
      for (int k = mn; k >= 1; --k) delta[k][j] = (c4 * delta[k][j] - k * delta[k - 1][j]) / c3;
      delta[0][j] = c4 * delta[0][j] / c3;
    }
    c1 = c2;
  }
}

bool make_colloc(int M, double dt, Colloc &co) {
  co = Colloc{};
  co.M = M;
  co.dt = dt;
  if (!radau_nodes(M, co.c)) return false;
  double prev = 0.0;
  for (int i = 0; i < M; ++i) {
    co.d[i] = co.c[i] - prev;
    prev = co.c[i];
  }
  long double x[MAXM];
  for (int i = 0; i < M; ++i) x[i] = co.c[i];
  std::vector<std::vector<long double>> delta;
  fornberg_weights(M, x, 0.0L, M - 1, delta);
  for (int k = 0; k < M; ++k)
    for (int j = 0; j < M; ++j) co.W[k][j] = (double)delta[k][j];
  co.invfact[0] = 1.0;
  for (int k = 1; k < MAXM + 10; ++k) co.invfact[k] = co.invfact[k - 1] / (double)k;
  for (int i = 0; i < M; ++i) {
    co.cpow[i][0] = 1.0;
    for (int k = 1; k <= M; ++k) co.cpow[i][k] = co.cpow[i][k - 1] * co.c[i];
  }
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      long double s = 0.0L;
      for (int k = 1; k <= M; ++k) s += (long double)co.cpow[i][k] * delta[k - 1][j] / (long double)std::tgamma(k + 1.0);
      co.Q[i][j] = (double)s;
    }
  return true;
}

// Row i of the result holds the Lagrange basis through c_from evaluated at
// c_to[i-1]; row 0 copies the start value (Sec. 3.2, R and T).
void transfer_matrix(int Mfrom, const double *c_from, int Mto, const double *c_to, double *out) {
  const int cols = Mfrom + 1;
  for (int i = 0; i <= Mto; ++i)
    for (int j = 0; j <= Mfrom; ++j) out[i * cols + j] = 0.0;
  out[0] = 1.0;
  for (int i = 1; i <= Mto; ++i) {
    const double s = c_to[i - 1];
    for (int j = 1; j <= Mfrom; ++j) {
      double l = 1.0;
      for (int m = 1; m <= Mfrom; ++m)
        if (m != j) l *= (s - c_from[m - 1]) / (c_from[j - 1] - c_from[m - 1]);
      out[i * cols + j] = l;
    }
  }
}

}  // namespace hsdc
