// Host: eigen-decomposition of small symmetric tridiagonal matrices for
// stochastic Lanczos quadrature, and of dense symmetric r x r matrices (the
// Nystrom preconditioner's spectral square root).
//
// Implicit symmetric QR iteration with the Wilkinson shift and bulge chasing
// by Givens rotations (Golub & Van Loan, Matrix Computations, Sec. 8.3), with
// deflation of negligible off-diagonal entries from the bottom.  Only the
// first component of every eigenvector is accumulated: the quadrature
// e_1^T f(T) e_1 = sum_m z_m^2 f(theta_m) needs nothing else.
#include <cmath>
#include <limits>
#include <vector>

#include "solver.h"

namespace gpk {

bool tridiag_eig_first(int n, double* a, double* b, double* z) {
  if (n <= 0) return false;
  for (int i = 0; i < n; ++i) z[i] = i == 0 ? 1.0 : 0.0;
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1;
  int sweeps = 0;
  while (hi > 0) {
    if (std::fabs(b[hi - 1]) <= eps * (std::fabs(a[hi - 1]) + std::fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(b[lo - 1]) > eps * (std::fabs(a[lo - 1]) + std::fabs(a[lo]))) --lo;
    if (++sweeps > 60 * n) return false;
    // Wilkinson shift: eigenvalue of the trailing 2x2 block closer to a[hi]
    const double dd = 0.5 * (a[hi - 1] - a[hi]);
    const double bb = b[hi - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, bb);
    const double mu = a[hi] - bb * bb / den;
    // chase the bulge from lo to hi
    double x = a[lo] - mu, y = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, y);
      const double c = r == 0.0 ? 1.0 : x / r;
      const double s = r == 0.0 ? 0.0 : y / r;
      if (k > lo) b[k - 1] = r;  // row k-1: (b_{k-1}, bulge) -> (r, 0)
      // rotate the 2x2 block [a_k b_k; b_k a_{k+1}]
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        // the rotation fills (k, k+2) with the new bulge
        y = s * b[k + 1];
        b[k + 1] = c * b[k + 1];
        x = b[k];
      }
      // first row of the accumulated eigenvector matrix
      const double zk = z[k], zk1 = z[k + 1];
      z[k] = c * zk + s * zk1;
      z[k + 1] = -s * zk + c * zk1;
    }
  }
  return true;
}

bool sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& Q) {
  // Householder reduction to tridiagonal form T = Q^T A Q (Golub & Van Loan, Sec. 8.3.1),
  // A row-major n x n, overwritten; Q accumulated explicitly.
  w.assign(n, 0.0);
  if (n <= 0) return false;
  std::vector<double> Qt((size_t)n * n, 0.0);  // Q^T: row j is column j of Q
  for (int i = 0; i < n; ++i) Qt[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), b(n > 1 ? n - 1 : 1, 0.0);
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += at(i, k) * at(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    const double x0 = at(k + 1, k);
    const double r = x0 >= 0.0 ? -alpha : alpha;  // new sub-diagonal entry
    // v = x - r e1, beta = 2 / v.v
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 - r;
    for (int i = k + 2; i < n; ++i) v[i] = at(i, k);
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // trailing block update A <- H A H with H = I - beta v v^T
    double pv = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += at(i, j) * v[j];
      p[i] = beta * acc;
      pv += p[i] * v[i];
    }
    const double half = 0.5 * beta * pv;
    for (int i = k + 1; i < n; ++i) p[i] -= half * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) at(i, j) -= v[i] * p[j] + p[i] * v[j];
    at(k + 1, k) = r;
    at(k, k + 1) = r;
    for (int i = k + 2; i < n; ++i) at(i, k) = at(k, i) = 0.0;
    // Q <- Q H, on Qt = Q^T (rows contiguous): Qt <- H Qt
    for (int i = 0; i < n; ++i) p[i] = 0.0;
    for (int j = k + 1; j < n; ++j) {
      const double* row = &Qt[(size_t)j * n];
      for (int i = 0; i < n; ++i) p[i] += v[j] * row[i];
    }
    for (int j = k + 1; j < n; ++j) {
      double* row = &Qt[(size_t)j * n];
      const double f = beta * v[j];
      for (int i = 0; i < n; ++i) row[i] -= f * p[i];
    }
  }
  for (int i = 0; i < n; ++i) w[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) b[i] = at(i + 1, i);
  // implicit symmetric QR on (w, b), the rotations accumulated into the columns of Q
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1, sweeps = 0;
  while (hi > 0) {
    if (std::fabs(b[hi - 1]) <= eps * (std::fabs(w[hi - 1]) + std::fabs(w[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(b[lo - 1]) > eps * (std::fabs(w[lo - 1]) + std::fabs(w[lo]))) --lo;
    if (++sweeps > 60 * n) return false;
    const double dd = 0.5 * (w[hi - 1] - w[hi]);
    const double bb = b[hi - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, bb);
    const double mu = w[hi] - bb * bb / den;
    double x = w[lo] - mu, y = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, y);
      const double c = r == 0.0 ? 1.0 : x / r;
      const double s = r == 0.0 ? 0.0 : y / r;
      if (k > lo) b[k - 1] = r;
      const double ak = w[k], ak1 = w[k + 1], bk = b[k];
      w[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      w[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        y = s * b[k + 1];
        b[k + 1] = c * b[k + 1];
        x = b[k];
      }
      double* q0 = &Qt[(size_t)k * n];
      double* q1 = &Qt[(size_t)(k + 1) * n];
      for (int i = 0; i < n; ++i) {
        const double t0 = q0[i], t1 = q1[i];
        q0[i] = c * t0 + s * t1;
        q1[i] = -s * t0 + c * t1;
      }
    }
  }
  Q.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + j] = Qt[(size_t)j * n + i];
  return true;
}

bool lanczos_log_quadrature(const double* alpha, const double* beta, int J, int stride, double* out) {
  if (J <= 0) {
    *out = 0.0;
    return true;
  }
  std::vector<double> a(J), b(J > 1 ? J - 1 : 1), z(J);
  for (int j = 0; j < J; ++j) {
    const double aj = alpha[(size_t)j * stride];
    if (!(aj > 0.0) || !std::isfinite(aj)) return false;
    a[j] = 1.0 / aj;
    if (j > 0) {
      const double bp = beta[(size_t)(j - 1) * stride];
      const double ap = alpha[(size_t)(j - 1) * stride];
      if (!(bp >= 0.0) || !std::isfinite(bp)) return false;
      a[j] += bp / ap;
      b[j - 1] = std::sqrt(bp) / ap;
    }
  }
  if (!tridiag_eig_first(J, a.data(), b.data(), z.data())) return false;
  double q = 0.0;
  for (int m = 0; m < J; ++m) {
    if (!(a[m] > 0.0)) return false;
    q += z[m] * z[m] * std::log(a[m]);
  }
  *out = q;
  return true;
}

}  // namespace gpk

extern "C" int gp_lanczos_quadrature(const double* alpha, const double* beta, int32_t J, int32_t stride,
                                     double* out) {
  if (!alpha || !beta || !out || J < 0 || stride < 1) return GP_EINVAL;
  return gpk::lanczos_log_quadrature(alpha, beta, J, stride, out) ? GP_OK : GP_ENOTPD;
}
