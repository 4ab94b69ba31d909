// Continued-fraction poles and residues of the Fermi function (Sec. II B, Eq. (7)).
//
// With y = x/2 the truncated fraction is f_M(x) = 1/2 - tanh_M(y)/2, and
// tanh_M(y) = y [(B + i y A)^{-1}]_{11} with B = diag(1, 3, ..., 2M-1) and A
// the M x M path matrix (zero diagonal, unit off-diagonals).  In the
// B-orthonormal eigenpairs of A v = lam B v this gives poles z = 2/lam and
// residues R = -v_0^2/lam^2 for each lam > 0.  The symmetric form
// C = B^{-1/2} A B^{-1/2} is tridiagonal with zero diagonal and off-diagonal
// 1/sqrt((2k-1)(2k+1)); u = B^{1/2} v, so v_0 = u_0.  C is diagonalised below
// by the implicit symmetric tridiagonal QR iteration with Wilkinson shifts
// (Golub and Van Loan, Sec. 8.3), accumulating the rotations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace ndrho {

// Eigen-decomposition of a symmetric tridiagonal matrix (diagonal a[n],
// off-diagonal b[n-1]).  On return a holds the eigenvalues and q (n x n,
// row-major, q[i*n+k] = component i of eigenvector k) the eigenvectors.
static void tridiag_qr(std::vector<double>& a, std::vector<double> b, std::vector<double>& q) {
  const int n = static_cast<int>(a.size());
  q.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) q[static_cast<size_t>(i) * n + i] = 1.0;
  if (n == 1) return;
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int sweeps = 0;
  while (hi > 0) {
    // deflate negligible off-diagonals
    for (int i = 0; i < hi; ++i) {
      if (std::fabs(b[i]) <= eps * (std::fabs(a[i]) + std::fabs(a[i + 1])) + 1e-300) b[i] = 0.0;
    }
    if (b[hi - 1] == 0.0) {
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && b[lo - 1] != 0.0) --lo;
    if (++sweeps > 100 * n) fail(NDRHO_EINVAL, "tridiagonal QR did not converge");
    // Wilkinson shift from the trailing 2x2 block
    const double d = 0.5 * (a[hi - 1] - a[hi]);
    const double bb = b[hi - 1];
    const double sgn = d >= 0.0 ? 1.0 : -1.0;
    const double mu = a[hi] - bb * bb / (d + sgn * std::hypot(d, bb));
    double x = a[lo] - mu;
    double z = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r;
      const double s = r == 0.0 ? 0.0 : z / r;
      if (k > lo) b[k - 1] = r;
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        z = s * b[k + 1];
        b[k + 1] = c * b[k + 1];
        x = b[k];
      }
      for (int i = 0; i < n; ++i) {
        double* row = &q[static_cast<size_t>(i) * n];
        const double qk = row[k], qk1 = row[k + 1];
        row[k] = c * qk + s * qk1;
        row[k + 1] = -s * qk + c * qk1;
      }
    }
  }
}

void cf_poles(int n_poles, double* z, double* r) {
  if (n_poles < 1) fail(NDRHO_EINVAL, "n_poles must be >= 1");
  const int m = 2 * n_poles;
  std::vector<double> a(m, 0.0), b(m - 1), q;
  for (int k = 1; k < m; ++k) b[k - 1] = 1.0 / std::sqrt((2.0 * k - 1.0) * (2.0 * k + 1.0));
  tridiag_qr(a, b, q);
  std::vector<std::pair<double, double>> zr;
  for (int k = 0; k < m; ++k) {
    const double lam = a[k];
    if (lam > 0.0) {
      const double u0 = q[k];  // row 0, column k
      zr.emplace_back(2.0 / lam, -(u0 * u0) / (lam * lam));
    }
  }
  if (static_cast<int>(zr.size()) != n_poles) fail(NDRHO_EINVAL, "unexpected number of positive eigenvalues");
  std::sort(zr.begin(), zr.end());
  for (int p = 0; p < n_poles; ++p) {
    z[p] = zr[p].first;
    r[p] = zr[p].second;
  }
}

}  // namespace ndrho
