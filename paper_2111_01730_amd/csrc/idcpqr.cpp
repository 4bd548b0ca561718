// Interpolative decomposition by column-pivoted Householder QR (eq. (ID), Section III-A).
//
// M P = Q R.  Keeping the first r pivot columns leaves the residual Q(:, r:) R22, whose
// Frobenius norm is the norm of the trailing block after r Householder steps, so the
// factorization stops at the first r with ||R22||_F <= chi ||M||_F.  Then
// V(:, P[:r]) = I and V(:, P[r:]) = R11^{-1} R12.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace hodbf {

int id_cpqr(cd *A, int m, int n, double chi, std::vector<int> &J, std::vector<cd> &V) {
  J.clear();
  V.clear();
  if (m <= 0 || n <= 0) return 0;
  std::vector<double> cn(n);
  double total2 = 0;
  for (int c = 0; c < n; ++c) {
    double s = 0;
    const cd *col = A + size_t(c) * m;
    for (int i = 0; i < m; ++i) s += std::norm(col[i]);
    cn[c] = s;
    total2 += s;
  }
  if (!(total2 > 0)) return 0;
  if (!std::isfinite(total2)) fail(HODBF_E_NUMERIC, "non-finite entries in an ID input");
  const double thr2 = chi * chi * total2;
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) piv[c] = c;
  const int k = std::min(m, n);
  int r = 0;
  std::vector<cd> u(m);
  for (int j = 0; j < k; ++j) {
    double trail = 0;
    for (int c = j; c < n; ++c) trail += cn[c];
    if (trail <= thr2) break;
    int p = j;
    for (int c = j + 1; c < n; ++c)
      if (cn[c] > cn[p]) p = c;  // first maximum on ties
    if (p != j) {
      std::swap_ranges(A + size_t(j) * m, A + size_t(j) * m + m, A + size_t(p) * m);
      std::swap(cn[j], cn[p]);
      std::swap(piv[j], piv[p]);
    }
    cd *x = A + size_t(j) * m;
    const int len = m - j;
    double xn2 = 0;
    for (int i = j; i < m; ++i) xn2 += std::norm(x[i]);
    const double xn = std::sqrt(xn2);
    const double aa = std::abs(x[j]);
    const cd phase = aa > 0 ? x[j] / aa : cd(1.0, 0.0);
    const cd beta = -phase * xn;  // reflector maps x(j:m) to beta e_1
    for (int i = 0; i < len; ++i) u[i] = x[j + i];
    u[0] -= beta;
    const double uu = 2.0 * xn * (xn + aa);  // u^H u
    if (uu > 0) {
      for (int c = j + 1; c < n; ++c) {
        cd *col = A + size_t(c) * m + j;
        cd s = 0;
        for (int i = 0; i < len; ++i) s += std::conj(u[i]) * col[i];
        s *= 2.0 / uu;
        for (int i = 0; i < len; ++i) col[i] -= u[i] * s;
      }
    }
    x[j] = beta;
    for (int i = j + 1; i < m; ++i) x[i] = 0;
    for (int c = j + 1; c < n; ++c) {
      const cd *col = A + size_t(c) * m;
      double s = 0;
      for (int i = j + 1; i < m; ++i) s += std::norm(col[i]);
      cn[c] = s;
    }
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
