// Interpolative decomposition by column-pivoted Householder QR (eq. (ID), Section III-A).
//
// M P = Q R.  Keeping the first r pivot columns leaves the residual Q(:, r:) R22, whose
// Frobenius norm is the norm of the trailing block after r Householder steps, so the
// factorization stops at the first r with ||R22||_F <= chi ||M||_F.  Then
// V(:, P[:r]) = I and V(:, P[r:]) = R11^{-1} R12.  The trailing column norms are
// downdated by each new row of R and recomputed whenever a norm has fallen below 5% of
// its last computed value (so cancellation never costs more than a few digits); the
// arithmetic runs on the real and imaginary parts.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace hodbf {

int id_cpqr(cd *A, int m, int n, double chi, std::vector<int> &J, std::vector<cd> &V) {
  J.clear();
  V.clear();
  if (m <= 0 || n <= 0) return 0;
  std::vector<double> cn(n), cn0(n);
  double total2 = 0;
  for (int c = 0; c < n; ++c) {
    double s = 0;
    const double *col = reinterpret_cast<const double *>(A + size_t(c) * m);
    for (int i = 0; i < 2 * m; ++i) s += col[i] * col[i];
    cn[c] = cn0[c] = s;
    total2 += s;
  }
  if (!(total2 > 0)) return 0;
  if (!std::isfinite(total2)) fail(HODBF_E_NUMERIC, "non-finite entries in an ID input");
  const double thr2 = chi * chi * total2;
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) piv[c] = c;
  const int k = std::min(m, n);
  int r = 0;
  std::vector<double> u(2 * size_t(m));
  for (int j = 0; j < k; ++j) {
    double trail = 0;
    for (int c = j; c < n; ++c) trail += cn[c];
    if (trail <= thr2) break;
    int p = j;
    for (int c = j + 1; c < n; ++c)
      if (cn[c] > cn[p]) p = c;
    if (p != j) {
      std::swap_ranges(A + size_t(j) * m, A + size_t(j) * m + m, A + size_t(p) * m);
      std::swap(cn[j], cn[p]);
      std::swap(cn0[j], cn0[p]);
      std::swap(piv[j], piv[p]);
    }
    double *x = reinterpret_cast<double *>(A + size_t(j) * m);
    const int len = m - j;
    double xn2 = 0;
    for (int i = 2 * j; i < 2 * m; ++i) xn2 += x[i] * x[i];
    const double xn = std::sqrt(xn2);
    const double aa = std::hypot(x[2 * j], x[2 * j + 1]);
    const double pr = aa > 0 ? x[2 * j] / aa : 1.0, pi = aa > 0 ? x[2 * j + 1] / aa : 0.0;
    const double br = -pr * xn, bi = -pi * xn;
    for (int i = 0; i < 2 * len; ++i) u[i] = x[2 * j + i];
    u[0] -= br;
    u[1] -= bi;
    const double uu = 2.0 * xn * (xn + aa);
    if (uu > 0) {
      const double f = 2.0 / uu;
      for (int c = j + 1; c < n; ++c) {
        double *col = reinterpret_cast<double *>(A + size_t(c) * m) + 2 * j;
        double sr = 0, si = 0;  // u^H col
        for (int i = 0; i < len; ++i) {
          sr += u[2 * i] * col[2 * i] + u[2 * i + 1] * col[2 * i + 1];
          si += u[2 * i] * col[2 * i + 1] - u[2 * i + 1] * col[2 * i];
        }
        sr *= f;
        si *= f;
        for (int i = 0; i < len; ++i) {
          col[2 * i] -= u[2 * i] * sr - u[2 * i + 1] * si;
          col[2 * i + 1] -= u[2 * i] * si + u[2 * i + 1] * sr;
        }
        // downdate the trailing norm by the new row-j entry; recompute when it has
        // lost most of its value (cancellation)
        const double rj2 = col[0] * col[0] + col[1] * col[1];
        cn[c] -= rj2;
        if (cn[c] <= 0.05 * cn0[c]) {
          double s = 0;
          for (int i = 2; i < 2 * len; ++i) s += col[i] * col[i];
          cn[c] = cn0[c] = s;
        }
      }
    } else {
      for (int c = j + 1; c < n; ++c) {
        const double *col = reinterpret_cast<const double *>(A + size_t(c) * m) + 2 * j;
        cn[c] -= col[0] * col[0] + col[1] * col[1];
      }
    }
    x[2 * j] = br;
    x[2 * j + 1] = bi;
    for (int i = 2 * (j + 1); i < 2 * m; ++i) x[i] = 0;
    r = j + 1;
  }
  J.assign(piv.begin(), piv.begin() + r);
  V.assign(size_t(r) * n, cd(0.0, 0.0));
  for (int c = 0; c < r; ++c) V[size_t(piv[c]) * r + c] = 1.0;
  std::vector<cd> t(r);
  for (int c = r; c < n; ++c) {
    const cd *col = A + size_t(c) * m;
    for (int i = r - 1; i >= 0; --i) {
      cd s = col[i];
      for (int l = i + 1; l < r; ++l) s -= A[size_t(l) * m + i] * t[l];
      t[i] = s / A[size_t(i) * m + i];
    }
    cd *vc = V.data() + size_t(piv[c]) * r;
    for (int i = 0; i < r; ++i) vc[i] = t[i];
  }
  return r;
}

}  // namespace hodbf
