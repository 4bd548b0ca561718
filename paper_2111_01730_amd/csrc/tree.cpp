// Cluster tree T_H by KD bisection (Section III-A) and host FP64 entries of Z.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace hodbf {

// Reading of "recursively subdividing the scatterer into two sub-scatterers with
// approximately equal numbers of unknowns using a tree clustering algorithm (such
// as KD)": split along the largest voxel-centre extent (ties x, then y, then z);
// the ceil(n/2) members lowest along that axis (ties by position) form the first
// child; both children keep their parent's order.  All nodes split to the same
// depth, the smallest L with ceil(N / 2^L) <= leaf_size.
Tree build_tree(int nx, int ny, int nz, int leaf_size) {
  Tree t;
  const int64_t n = int64_t(nx) * ny * nz;
  t.n = n;
  int L = 0;
  while ((n + (int64_t(1) << L) - 1) >> L > leaf_size) ++L;
  if (L > 0 && n < (int64_t(1) << L)) fail(HODBF_E_ARG, "grid too small for a complete tree");
  t.depth = L;
  std::vector<int32_t> cur(n), nxt(n);
  for (int64_t i = 0; i < n; ++i) cur[i] = int32_t(i);
  auto coord = [&](int32_t u, int axis) -> int {
    if (axis == 0) return u % nx;
    if (axis == 1) return (u / nx) % ny;
    return u / (nx * ny);
  };
  t.lo.assign(L + 1, {});
  t.lo[0] = {0, int32_t(n)};
  std::vector<int64_t> count(std::max({nx, ny, nz}) + 1);
  for (int l = 0; l < L; ++l) {
    const auto &plo = t.lo[l];
    auto &clo = t.lo[l + 1];
    clo.assign((size_t(1) << (l + 1)) + 1, 0);
    for (size_t i = 0; i + 1 < plo.size(); ++i) {
      const int32_t a = plo[i], b = plo[i + 1];
      const int32_t sz = b - a;
      int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-1, -1, -1};
      for (int32_t k = a; k < b; ++k)
        for (int ax = 0; ax < 3; ++ax) {
          int c = coord(cur[k], ax);
          mn[ax] = std::min(mn[ax], c);
          mx[ax] = std::max(mx[ax], c);
        }
      int axis = 0;
      for (int ax = 1; ax < 3; ++ax)
        if (mx[ax] - mn[ax] > mx[axis] - mn[axis]) axis = ax;
      const int32_t n1 = (sz + 1) / 2;
      std::fill(count.begin(), count.end(), 0);
      for (int32_t k = a; k < b; ++k) count[coord(cur[k], axis)]++;
      int thr = 0;
      int64_t below = 0;  // members with coordinate < thr
      while (below + count[thr] < n1) below += count[thr++];
      int64_t ties_first = n1 - below;  // members at coordinate thr that go first
      int32_t w1 = a, w2 = a + n1;
      for (int32_t k = a; k < b; ++k) {
        const int c = coord(cur[k], axis);
        const bool first = c < thr || (c == thr && ties_first-- > 0);
        if (first) nxt[w1++] = cur[k];
        else nxt[w2++] = cur[k];
      }
      clo[2 * i] = a;
      clo[2 * i + 1] = a + n1;
      clo[2 * i + 2] = b;
    }
    std::swap(cur, nxt);
  }
  t.perm = cur;
  t.cx.resize(n);
  t.cy.resize(n);
  t.cz.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    t.cx[i] = int16_t(coord(cur[i], 0));
    t.cy[i] = int16_t(coord(cur[i], 1));
    t.cz[i] = int16_t(coord(cur[i], 2));
  }
  return t;
}

Kernel make_kernel(const Tree &t, const std::vector<cd> &eps_user, double h, double k0) {
  Kernel k;
  k.tree = &t;
  k.kh = k0 * h;
  k.ka = k0 * h * std::cbrt(3.0 / (4.0 * M_PI));
  // k^2 S(a): the Green's function integrated over the equal-volume sphere
  k.k2S = cd(1.0, k.ka) * std::exp(cd(0.0, -k.ka)) - 1.0;
  k.inv_eps.resize(t.n);
  k.kappa.resize(t.n);
  for (int64_t i = 0; i < t.n; ++i) {
    const cd e = eps_user[t.perm[i]];
    k.inv_eps[i] = 1.0 / e;
    k.kappa[i] = (e - 1.0) / e;
  }
  return k;
}

cd Kernel::entry(int32_t m, int32_t n) const {
  const Tree &t = *tree;
  const int dx = t.cx[m] - t.cx[n], dy = t.cy[m] - t.cy[n], dz = t.cz[m] - t.cz[n];
  const int d2 = dx * dx + dy * dy + dz * dz;
  if (d2 == 0) return inv_eps[m] - k2S * kappa[n];
  const double rho = std::sqrt(double(d2));
  const double s = kh * kh / (4.0 * M_PI * rho);
  const double ph = kh * rho;
  return -cd(s * std::cos(ph), -s * std::sin(ph)) * kappa[n];
}

}  // namespace hodbf
