// Algorithm 1 (HODBF_invert) and Algorithm 2 (BF_SMW) of Section III-B, with every new
// butterfly reconstructed from products with structured random vectors
// (BF_random_matvec), written once over the Engine / LinOp interfaces of construct.h.
#include "construct.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <set>

namespace hodbf {

namespace {

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// composite operators
class Chain final : public LinOp {
 public:
  explicit Chain(std::vector<OpP> ops) : ops_(std::move(ops)) {}
  void apply(Engine &E, bool trans, const Mv &x, Mv &y) const override {
    const int n = int(ops_.size());
    if (n == 1) {
      ops_[0]->apply(E, trans, x, y);
      return;
    }
    MvP a = E.make(x.R), b = E.make(x.R);
    const Mv *cur = &x;
    for (int i = 0; i < n; ++i) {
      const LinOp &op = *ops_[size_t(trans ? n - 1 - i : i)];
      Mv &dst = i == n - 1 ? y : (i % 2 == 0 ? *a : *b);
      op.apply(E, trans, *cur, dst);
      cur = &dst;
    }
  }

 private:
  std::vector<OpP> ops_;
};

class LinComb final : public LinOp {
 public:
  explicit LinComb(std::vector<std::pair<cd, OpP>> t) : t_(std::move(t)) {}
  void apply(Engine &E, bool trans, const Mv &x, Mv &y) const override {
    E.zero(y);
    MvP tmp;
    for (const auto &[c, op] : t_) {
      if (!op) {
        E.axpy(c, x, y);
        continue;
      }
      if (!tmp) tmp = E.make(x.R);
      op->apply(E, trans, x, *tmp);
      E.axpy(c, *tmp, y);
    }
  }

 private:
  std::vector<std::pair<cd, OpP>> t_;
};

class PlusI final : public LinOp {
 public:
  explicit PlusI(OpP F) : F_(std::move(F)) {}
  void apply(Engine &E, bool trans, const Mv &x, Mv &y) const override {
    F_->apply(E, trans, x, y);
    E.axpy(1.0, x, y);
  }

 private:
  OpP F_;
};

class Mask final : public LinOp {
 public:
  explicit Mask(RowSet r) : r_(std::move(r)) {}
  void apply(Engine &E, bool, const Mv &x, Mv &y) const override {
    E.copy(x, y);
    E.keep_rows(r_, y);
  }

 private:
  RowSet r_;
};

// z = leaf x, then z += F z for each level operator (towards the root).
class MulInv final : public LinOp {
 public:
  MulInv(OpP leaf, std::vector<OpP> lv) : leaf_(std::move(leaf)), lv_(std::move(lv)) {}
  void apply(Engine &E, bool trans, const Mv &x, Mv &y) const override {
    MvP t = E.make(x.R);
    if (!trans) {
      leaf_->apply(E, false, x, y);
      for (const OpP &F : lv_) {
        F->apply(E, false, y, *t);
        E.axpy(1.0, *t, y);
      }
      return;
    }
    MvP z = E.make(x.R);
    E.copy(x, *z);
    for (auto it = lv_.rbegin(); it != lv_.rend(); ++it) {
      (*it)->apply(E, true, *z, *t);
      E.axpy(1.0, *t, *z);
    }
    leaf_->apply(E, true, *z, y);
  }

 private:
  OpP leaf_;
  std::vector<OpP> lv_;
};

// F = A^{-1} - I for A = [I + E11, E12; E21, I + E22] on every node of a set, from
// F11 = (I + E11 - E12 (I + F22) E21)^{-1} - I and F22 = (I + E22)^{-1} - I:
//   A^{-1} = [I, 0; -(I+F22) E21, I] diag(I + F11, I + F22) [I, -E12 (I+F22); 0, I]
// (the product of Algorithm 2's last step).  P1 / P2: the rows of the first / second
// children of the nodes.
class SmwProduct final : public LinOp {
 public:
  SmwProduct(OpP E12, OpP E21, OpP F11, OpP F22, RowSet P1, RowSet P2)
      : E12_(std::move(E12)), E21_(std::move(E21)), F11_(std::move(F11)), F22_(std::move(F22)),
        P1_(std::move(P1)), P2_(std::move(P2)) {}
  void apply(Engine &E, bool trans, const Mv &x, Mv &y) const override {
    const int R = x.R;
    MvP x1 = E.make(R), x2 = E.make(R), t = E.make(R), u = E.make(R), v = E.make(R);
    E.copy(x, *x1);
    E.keep_rows(P1_, *x1);
    E.copy(x, *x2);
    E.keep_rows(P2_, *x2);
    // v = (I + F22)^(T) x2
    E.copy(*x2, *v);
    if (F22_) {
      F22_->apply(E, trans, *x2, *t);
      E.axpy(1.0, *t, *v);
    }
    if (!trans) {
      // w = x1 - E12 v ; y1 = (I + F11) w ; y2 = v - (I + F22) E21 y1
      MvP w = E.make(R);
      E.copy(*x1, *w);
      if (E12_) {
        E12_->apply(E, false, *v, *t);
        E.axpy(-1.0, *t, *w);
      }
      MvP y1 = E.make(R);
      E.copy(*w, *y1);
      if (F11_) {
        F11_->apply(E, false, *w, *t);
        E.axpy(1.0, *t, *y1);
      }
      E.copy(*v, *u);  // u = y2
      if (E21_) {
        E21_->apply(E, false, *y1, *t);
        E.axpy(-1.0, *t, *u);
        if (F22_) {
          MvP s = E.make(R);
          F22_->apply(E, false, *t, *s);
          E.axpy(-1.0, *s, *u);
        }
      }
      // y = (y1 - x1) + (y2 - x2)
      E.copy(*y1, y);
      E.axpy(-1.0, *x1, y);
      E.axpy(1.0, *u, y);
      E.axpy(-1.0, *x2, y);
      return;
    }
    // transposed: a1 = x1 - E21^T v ; b1 = (I + F11)^T a1 ; c2 = v - (I + F22)^T E12^T b1
    MvP a1 = E.make(R);
    E.copy(*x1, *a1);
    if (E21_) {
      E21_->apply(E, true, *v, *t);
      E.axpy(-1.0, *t, *a1);
    }
    MvP b1 = E.make(R);
    E.copy(*a1, *b1);
    if (F11_) {
      F11_->apply(E, true, *a1, *t);
      E.axpy(1.0, *t, *b1);
    }
    E.copy(*v, *u);  // u = c2
    if (E12_) {
      E12_->apply(E, true, *b1, *t);
      E.axpy(-1.0, *t, *u);
      if (F22_) {
        MvP s = E.make(R);
        F22_->apply(E, true, *t, *s);
        E.axpy(-1.0, *s, *u);
      }
    }
    E.copy(*b1, y);
    E.axpy(-1.0, *x1, y);
    E.axpy(1.0, *u, y);
    E.axpy(-1.0, *x2, y);
  }

 private:
  OpP E12_, E21_, F11_, F22_;
  RowSet P1_, P2_;
};

// ---------------------------------------------------------------------------
// small dense helpers (complex FP64, column-major)

// In-place inverse by Gauss-Jordan elimination with partial pivoting (row interchanges,
// undone as column interchanges in reverse order at the end).  Column-major; each
// elimination step is a rank-1 update whose inner loop runs down a contiguous column,
// written on the real and imaginary parts.
void inverse_inplace(std::vector<cd> &A, int n) {
  std::vector<int> piv(static_cast<size_t>(n));
  std::vector<double> mc(2 * static_cast<size_t>(n));
  double *a = reinterpret_cast<double *>(A.data());
  for (int c = 0; c < n; ++c) {
    double *colc = a + 2 * size_t(c) * n;
    int p = c;
    double best = std::hypot(colc[2 * c], colc[2 * c + 1]);
    for (int r = c + 1; r < n; ++r) {
      const double v = std::hypot(colc[2 * r], colc[2 * r + 1]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    if (!(best > 0) || !std::isfinite(best)) fail(HODBF_E_NUMERIC, "singular block in the preconditioner");
    piv[size_t(c)] = p;
    if (p != c)
      for (int k = 0; k < n; ++k) {
        double *col = a + 2 * size_t(k) * n;
        std::swap(col[2 * p], col[2 * c]);
        std::swap(col[2 * p + 1], col[2 * c + 1]);
      }
    // d = 1 / A(c, c); the old column c is kept as the multipliers
    const double pr = colc[2 * c], pi = colc[2 * c + 1], den = pr * pr + pi * pi;
    const double dr = pr / den, di = -pi / den;
    std::copy(colc, colc + 2 * size_t(n), mc.data());
    for (int k = 0; k < n; ++k) {
      if (k == c) continue;
      double *col = a + 2 * size_t(k) * n;
      const double fr = col[2 * c] * dr - col[2 * c + 1] * di;
      const double fi = col[2 * c] * di + col[2 * c + 1] * dr;
      if (fr != 0 || fi != 0)
        for (int r = 0; r < n; ++r) {
          col[2 * r] -= mc[2 * size_t(r)] * fr - mc[2 * size_t(r) + 1] * fi;
          col[2 * r + 1] -= mc[2 * size_t(r)] * fi + mc[2 * size_t(r) + 1] * fr;
        }
      col[2 * c] = fr;
      col[2 * c + 1] = fi;
    }
    for (int r = 0; r < n; ++r) {
      const double mr = mc[2 * size_t(r)], mi = mc[2 * size_t(r) + 1];
      colc[2 * r] = -(mr * dr - mi * di);
      colc[2 * r + 1] = -(mr * di + mi * dr);
    }
    colc[2 * c] = dr;
    colc[2 * c + 1] = di;
  }
  for (int c = n - 1; c >= 0; --c) {
    const int p = piv[size_t(c)];
    if (p != c)
      std::swap_ranges(a + 2 * size_t(c) * n, a + 2 * size_t(c + 1) * n, a + 2 * size_t(p) * n);
  }
}

// X (n x nrhs) minimizing ||A X - B||_F, A m x n, B m x nrhs (column-major), by
// Householder QR with column pivoting; directions below 1e-13 of the largest are dropped.
std::vector<cd> lstsq(std::vector<cd> A, int m, int n, std::vector<cd> B, int nrhs) {
  std::vector<cd> X(static_cast<size_t>(n) * nrhs, cd(0, 0));
  if (m == 0 || n == 0 || nrhs == 0) return X;
  std::vector<int> piv(n);
  for (int c = 0; c < n; ++c) piv[c] = c;
  // trailing column norms, downdated by each new row of R and recomputed once one has
  // fallen below 5% of its last computed value
  std::vector<double> cn(n), cn0(n);
  for (int c = 0; c < n; ++c) {
    double s = 0;
    const double *col = reinterpret_cast<const double *>(A.data() + size_t(c) * m);
    for (int i = 0; i < 2 * m; ++i) s += col[i] * col[i];
    cn[c] = cn0[c] = s;
  }
  const int kmax = std::min(m, n);
  int r = 0;
  double top = 0;
  std::vector<double> u(2 * size_t(m));
  for (int j = 0; j < kmax; ++j) {
    int p = j;
    for (int c = j + 1; c < n; ++c)
      if (cn[c] > cn[p]) p = c;
    if (p != j) {
      std::swap_ranges(A.begin() + size_t(j) * m, A.begin() + size_t(j) * m + m, A.begin() + size_t(p) * m);
      std::swap(cn[j], cn[p]);
      std::swap(cn0[j], cn0[p]);
      std::swap(piv[j], piv[p]);
    }
    double *x = reinterpret_cast<double *>(A.data() + size_t(j) * m);
    double xn2 = 0;
    for (int i = 2 * j; i < 2 * m; ++i) xn2 += x[i] * x[i];
    const double xn = std::sqrt(xn2);
    if (j == 0) top = xn;
    if (!(xn > 1e-13 * top)) break;
    const double aa = std::hypot(x[2 * j], x[2 * j + 1]);
    const double pr = aa > 0 ? x[2 * j] / aa : 1.0, pi = aa > 0 ? x[2 * j + 1] / aa : 0.0;
    const double br = -pr * xn, bi = -pi * xn;  // the reflector maps x(j:m) to beta e_1
    const int len = m - j;
    for (int i = 0; i < 2 * len; ++i) u[i] = x[2 * j + i];
    u[0] -= br;
    u[1] -= bi;
    const double f = 2.0 / (2.0 * xn * (xn + aa));  // 2 / u^H u
    auto reflect = [&](cd *column) {
      double *col = reinterpret_cast<double *>(column) + 2 * j;
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
      return col;
    };
    for (int c = j + 1; c < n; ++c) {
      const double *col = reflect(A.data() + size_t(c) * m);
      cn[c] -= col[0] * col[0] + col[1] * col[1];
      if (cn[c] <= 0.05 * cn0[c]) {
        double s2 = 0;
        for (int i = 2; i < 2 * len; ++i) s2 += col[i] * col[i];
        cn[c] = cn0[c] = s2;
      }
    }
    for (int c = 0; c < nrhs; ++c) reflect(B.data() + size_t(c) * m);
    x[2 * j] = br;
    x[2 * j + 1] = bi;
    for (int i = 2 * (j + 1); i < 2 * m; ++i) x[i] = 0;
    r = j + 1;
  }
  std::vector<cd> t(r);
  for (int q = 0; q < nrhs; ++q) {
    for (int i = r - 1; i >= 0; --i) {
      cd s = B[size_t(q) * m + i];
      for (int l = i + 1; l < r; ++l) s -= A[size_t(l) * m + i] * t[l];
      t[i] = s / A[size_t(i) * m + i];
    }
    for (int i = 0; i < r; ++i) X[size_t(q) * n + piv[i]] = t[i];
  }
  return X;
}

// C = A B (A m x k, B k x n, column-major, complex FP64)
std::vector<cd> matmul(const std::vector<cd> &A, int m, int k, const std::vector<cd> &B, int n) {
  std::vector<cd> C(static_cast<size_t>(m) * n, cd(0, 0));
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      const cd b = B[size_t(j) * k + l];
      if (b == cd(0, 0)) continue;
      const cd *a = A.data() + size_t(l) * m;
      cd *c = C.data() + size_t(j) * m;
      for (int i = 0; i < m; ++i) c[i] += a[i] * b;
    }
  return C;
}

std::vector<cd> to_cd(const Mat &M) { return std::vector<cd>(M.v.begin(), M.v.end()); }
Mat to_mat(const std::vector<cd> &v, int m, int n) {
  Mat M;
  M.m = m;
  M.n = n;
  M.v.assign(v.begin(), v.end());
  return M;
}

uint64_t mix(uint64_t a, uint64_t b) {
  uint64_t z = a + 0x9E3779B97F4A7C15ull * (b + 1);
  z ^= z >> 31;
  z *= 0xD6E8FEB86659FD93ull;
  z ^= z >> 29;
  return z;
}

void drop_cols(Mat &f, int c0, int cnt) {
  if (cnt == 0) return;
  std::vector<cf> nv;
  if (f.m > 0) {
    nv.reserve(size_t(f.m) * size_t(f.n - cnt));
    for (int k = 0; k < f.n; ++k) {
      if (k >= c0 && k < c0 + cnt) continue;
      nv.insert(nv.end(), f.v.begin() + size_t(k) * f.m, f.v.begin() + size_t(k + 1) * f.m);
    }
  }
  f.v.swap(nv);
  f.n -= cnt;
}

// rank (output rows) of block idx at stage s (0: V^0)
Mat &stage_block(Butterfly &bf, int s, int64_t idx) {
  return s == 0 ? bf.V0[size_t(idx)] : bf.W[size_t(s)][size_t(idx)];
}

// Remove the rows of stage block (s, (a, b)) and the matching columns of its readers.
void drop_rows(Butterfly &bf, int s, int64_t a, int64_t b) {
  const int L = bf.L;
  const int64_t nb = int64_t(1) << (L - s);
  Mat &w = stage_block(bf, s, a * nb + b);
  const int m = w.m;
  if (m == 0) return;
  w.m = 0;
  w.v.clear();
  if (s == L) {
    drop_cols(bf.B[size_t(a)], 0, m);
    return;
  }
  const int64_t nb2 = nb / 2;
  const int first = (b & 1) ? stage_block(bf, s, a * nb + (b & ~int64_t(1))).m : 0;
  for (int c = 0; c < 2; ++c) {
    Mat &f = bf.W[size_t(s + 1)][size_t((2 * a + c) * nb2 + b / 2)];
    if (f.n >= first + m) drop_cols(f, first, m);
  }
}

}  // namespace

// Keep every stage row both written and read: a transfer block that reads nothing
// (its inputs all have rank 0) outputs zeros, and a stage output that no later block
// reads is dead; both lose their rows (and the matching columns downstream), until
// nothing changes.  The product is unchanged.
void prune_butterfly(Butterfly &bf) {
  const int L = bf.L;
  for (bool changed = true; changed;) {
    changed = false;
    for (int s = 1; s <= L; ++s) {
      const int64_t na = int64_t(1) << s, nb = int64_t(1) << (L - s);
      for (int64_t a = 0; a < na; ++a)
        for (int64_t b = 0; b < nb; ++b) {
          const Mat &w = bf.W[size_t(s)][size_t(a * nb + b)];
          if (w.m > 0 && w.n == 0) {
            drop_rows(bf, s, a, b);
            changed = true;
          }
        }
    }
    for (int s = 0; s < L; ++s) {
      const int64_t na = int64_t(1) << s, nb = int64_t(1) << (L - s);
      for (int64_t a = 0; a < na; ++a)
        for (int64_t b = 0; b < nb; ++b) {
          if (stage_block(bf, s, a * nb + b).m == 0) continue;
          const int64_t nb2 = nb / 2;
          bool read = false;
          for (int c = 0; c < 2; ++c)
            read = read || bf.W[size_t(s + 1)][size_t((2 * a + c) * nb2 + b / 2)].m > 0;
          if (!read) {
            drop_rows(bf, s, a, b);
            changed = true;
          }
        }
    }
  }
}

OpP chain(std::vector<OpP> ops) { return std::make_shared<Chain>(std::move(ops)); }
OpP lincomb(std::vector<std::pair<cd, OpP>> t) { return std::make_shared<LinComb>(std::move(t)); }
OpP plus_identity(OpP F) { return std::make_shared<PlusI>(std::move(F)); }
OpP row_mask(RowSet rows) { return std::make_shared<Mask>(std::move(rows)); }
OpP mult_inverse(Engine &, OpP leaf, const std::vector<OpP> &levels) {
  return std::make_shared<MulInv>(std::move(leaf), levels);
}

// ---------------------------------------------------------------------------
// randomized reconstruction of a set of butterflies (the BF_random_matvec step)

namespace {

struct SideLevel {
  std::vector<std::vector<std::vector<int32_t>>> skel;  // [target][pair]
  std::vector<std::vector<Mat>> fac;                     // [target][pair]: r x nc
  std::vector<std::vector<std::vector<cd>>> gsel;        // row side, middle level: k x r
  int k = 0;
  uint64_t seed = 0;
};

// rank of the value among the sorted distinct values of a list
int rank_in(std::vector<int64_t> v, int64_t x) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return int(std::lower_bound(v.begin(), v.end(), x) - v.begin());
}

}  // namespace

std::vector<Butterfly> reconstruct(Engine &E, const LinOp &M, int lev, int L,
                                   const std::vector<Target> &tg, const RbfOpts &o,
                                   RbfStats *st) {
  const Tree &t = *E.tree;
  const int T = int(tg.size());
  const int ll = lev + L;
  if (ll > t.depth) fail(HODBF_E_ARG, "reconstruction below the leaves of the tree");
  const int h = L / 2;
  // classes: targets sharing a column node but differing in row node must not share
  // sketch columns on the column side (and vice versa), or their sketches would mix
  std::vector<int> clsC(static_cast<size_t>(T)), clsR(static_cast<size_t>(T));
  int nclsC = 1, nclsR = 1;
  for (int b = 0; b < T; ++b) {
    std::vector<int64_t> os, ss;
    for (int c = 0; c < T; ++c) {
      if (tg[size_t(c)].si == tg[size_t(b)].si) os.push_back(tg[size_t(c)].oi);
      if (tg[size_t(c)].oi == tg[size_t(b)].oi) ss.push_back(tg[size_t(c)].si);
    }
    clsC[size_t(b)] = rank_in(os, tg[size_t(b)].oi);
    clsR[size_t(b)] = rank_in(ss, tg[size_t(b)].si);
    nclsC = std::max(nclsC, clsC[size_t(b)] + 1);
    nclsR = std::max(nclsR, clsR[size_t(b)] + 1);
  }
  const uint64_t seed0 = mix(mix(o.seed, uint64_t(lev)), uint64_t(L) + 1000 * uint64_t(T));
  std::vector<SideLevel> C(static_cast<size_t>(h + 1)), Rw(size_t(L - h + 1));
  int k_cur[2] = {o.k0_side[0] > 0 ? o.k0_side[0] : o.k0, o.k0_side[1] > 0 ? o.k0_side[1] : o.k0};

  // one sweep level of one side: sketch, gather the candidates of every pair, ID them
  auto sweep = [&](bool colside, int j, int kmin) {
    std::vector<SideLevel> &S = colside ? C : Rw;
    SideLevel &cur = S[size_t(j)];
    const int nsup = 1 << j, ncand = 1 << (L - j);
    const int npair = nsup * ncand;
    const int ncls = colside ? nclsC : nclsR;
    const int nslot = ncls * nsup;
    std::vector<int32_t> slot_of_row(static_cast<size_t>(t.n), -1);
    for (int b = 0; b < T; ++b) {
      const int64_t top = colside ? tg[size_t(b)].oi : tg[size_t(b)].si;
      const int cls = colside ? clsC[size_t(b)] : clsR[size_t(b)];
      for (int a = 0; a < nsup; ++a) {
        const int64_t node = (top << j) + a;
        const int32_t slot = cls * nsup + a;
        for (int32_t r = t.node_lo(lev + j, node); r < t.node_hi(lev + j, node); ++r) {
          int32_t &s = slot_of_row[size_t(r)];
          if (s >= 0 && s != slot) fail(HODBF_E_ARG, "reconstruction targets overlap in a sketch slot");
          s = slot;
        }
      }
    }
    // candidates of every (target, pair)
    std::vector<std::vector<std::vector<int32_t>>> cand(static_cast<size_t>(T), std::vector<std::vector<int32_t>>(size_t(npair)));
    for (int b = 0; b < T; ++b) {
      const int64_t ctop = colside ? tg[size_t(b)].si : tg[size_t(b)].oi;
      for (int a = 0; a < nsup; ++a)
        for (int c = 0; c < ncand; ++c) {
          auto &cl = cand[size_t(b)][size_t(a * ncand + c)];
          if (j == 0) {
            const int64_t node = (ctop << L) + c;
            for (int32_t r = t.node_lo(ll, node); r < t.node_hi(ll, node); ++r) cl.push_back(r);
          } else {
            const SideLevel &pv = S[size_t(j - 1)];
            const int64_t pp = int64_t(a / 2) * (2 * ncand) + 2 * c;
            const auto &s1 = pv.skel[size_t(b)][size_t(pp)];
            const auto &s2 = pv.skel[size_t(b)][size_t(pp + 1)];
            cl.insert(cl.end(), s1.begin(), s1.end());
            cl.insert(cl.end(), s2.begin(), s2.end());
          }
        }
    }
    int k = std::max(k_cur[colside ? 0 : 1], kmin);
    k = std::min(k, o.kmax);
    for (int attempt = 0;; ++attempt) {
      const uint64_t seed = mix(seed0, uint64_t(colside ? 1 : 2) * 1000003ull + uint64_t(j) * 131ull + uint64_t(attempt));
      // gathered sketch blocks per (target, pair): k x nc column-major
      std::vector<std::vector<std::vector<cd>>> G(static_cast<size_t>(T), std::vector<std::vector<cd>>(size_t(npair)));
      const int spc = std::max(1, E.max_cols() / k);
      for (int s0 = 0; s0 < nslot; s0 += spc) {
        const int s1 = std::min(nslot, s0 + spc);
        const int R = (s1 - s0) * k;
        auto t0 = std::chrono::steady_clock::now();
        MvP X = E.make(R);
        E.fill_sketch(*X, slot_of_row, int64_t(s0) * k, k, seed);
        MvP Y = E.make(R);
        M.apply(E, colside, *X, *Y);
        std::vector<Gather> req;
        std::vector<std::pair<int, int>> who;
        for (int b = 0; b < T; ++b) {
          const int cls = colside ? clsC[size_t(b)] : clsR[size_t(b)];
          for (int a = 0; a < nsup; ++a) {
            const int slot = cls * nsup + a;
            if (slot < s0 || slot >= s1) continue;
            for (int c = 0; c < ncand; ++c) {
              const int p = a * ncand + c;
              if (cand[size_t(b)][size_t(p)].empty()) continue;
              req.push_back({int32_t((slot - s0) * k), cand[size_t(b)][size_t(p)]});
              who.push_back({b, p});
            }
          }
        }
        std::vector<cd> out;
        E.gather(*Y, req, k, out);
        size_t off = 0;
        for (size_t q = 0; q < req.size(); ++q) {
          const size_t cnt = req[q].rows.size() * size_t(k);
          G[size_t(who[q].first)][size_t(who[q].second)].assign(out.begin() + off, out.begin() + off + cnt);
          off += cnt;
        }
        if (st) {
          st->sketch_cols += R;
          st->applies += 1;
          st->seconds_apply += seconds_since(t0);
        }
      }
      auto th = std::chrono::steady_clock::now();
      cur.skel.assign(size_t(T), std::vector<std::vector<int32_t>>(size_t(npair)));
      cur.fac.assign(size_t(T), std::vector<Mat>(size_t(npair)));
      const bool keep = !colside && j == L - h;
      if (keep) cur.gsel.assign(size_t(T), std::vector<std::vector<cd>>(size_t(npair)));
      int saturated = 0, maxr = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : saturated) reduction(max : maxr)
      for (int64_t q = 0; q < int64_t(T) * npair; ++q) {
        const int b = int(q / npair), p = int(q % npair);
        const auto &cl = cand[size_t(b)][size_t(p)];
        const int nc = int(cl.size());
        Mat f;
        f.n = nc;
        if (nc > 0) {
          std::vector<cd> A = G[size_t(b)][size_t(p)];
          std::vector<int> J;
          std::vector<cd> V;
          const int r = id_cpqr(A.data(), k, nc, o.chi, J, V);
          if (r > k - o.oversample && r < nc) ++saturated;
          maxr = std::max(maxr, r);
          f.m = r;
          f.v.assign(V.begin(), V.end());
          auto &sk = cur.skel[size_t(b)][size_t(p)];
          sk.resize(size_t(r));
          for (int i = 0; i < r; ++i) sk[size_t(i)] = cl[size_t(J[size_t(i)])];
          if (keep) {
            auto &gs = cur.gsel[size_t(b)][size_t(p)];
            gs.resize(size_t(k) * size_t(r));
            const auto &g = G[size_t(b)][size_t(p)];
            for (int i = 0; i < r; ++i)
              std::copy(g.begin() + size_t(J[size_t(i)]) * k, g.begin() + size_t(J[size_t(i)] + 1) * k,
                        gs.begin() + size_t(i) * k);
          }
        }
        cur.fac[size_t(b)][size_t(p)] = std::move(f);
      }
      if (st) {
        st->ids += int64_t(T) * npair;
        st->seconds_id += seconds_since(th);
        st->max_rank = std::max(st->max_rank, maxr);
      }
      if (saturated && k < o.kmax) {
        if (st) ++st->redone;
        logf("    sketch width %d saturated (%d blocks, rank %d) at %s level %d; doubling", k,
             saturated, maxr, colside ? "column" : "row", j);
        k = std::min(2 * k, o.kmax);
        continue;
      }
      cur.k = k;
      cur.seed = seed;
      k_cur[colside ? 0 : 1] = k;
      break;
    }
  };

  for (int j = 0; j <= h; ++j) sweep(true, j, 0);
  // the middle fit needs every column-side rank below the row side's last sketch width
  int max_rc = 0;
  for (const auto &tb : C[size_t(h)].skel)
    for (const auto &s : tb) max_rc = std::max(max_rc, int(s.size()));
  for (int j = 0; j <= L - h; ++j) sweep(false, j, j == L - h ? max_rc + o.oversample : 0);
  if (st) {
    st->last_k[0] = k_cur[0];
    st->last_k[1] = k_cur[1];
  }

  // middle: S_{tau,nu} (r_r x r_c) with X_nu(rows tau_bar, :) ~ S (V_{tau,nu} Omega_nu),
  // V_{tau,nu} Omega_nu propagated through the column-side factors on the host
  auto tm = std::chrono::steady_clock::now();
  const int nt = 1 << h, nn = 1 << (L - h);
  const SideLevel &RL = Rw[size_t(L - h)];
  std::vector<std::vector<Mat>> S(static_cast<size_t>(T), std::vector<Mat>(size_t(nt) * nn));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < int64_t(T) * nn; ++q) {
    const int b = int(q / nn), nu = int(q % nn);
    const int kR = RL.k;
    const int64_t slot = int64_t(clsR[size_t(b)]) * nn + nu;
    const int64_t nu_node = (tg[size_t(b)].si << (L - h)) + nu;
    const int32_t nu_lo = t.node_lo(ll - h, nu_node);
    // level 0 of the cone: every leaf of T_s under nu
    std::vector<std::vector<cd>> tv(static_cast<size_t>(1) << h);  // per (tau', nu') of the current level
    for (int c0 = 0; c0 < (1 << h); ++c0) {
      const int64_t leaf = int64_t(nu) * (1 << h) + c0;
      const Mat &V = C[0].fac[size_t(b)][size_t(leaf)];
      const int64_t node = (tg[size_t(b)].si << L) + leaf;
      const int32_t lo = t.node_lo(ll, node), hi = t.node_hi(ll, node);
      const int nr = hi - lo;
      std::vector<cd> Om(static_cast<size_t>(nr) * kR);
      for (int qq = 0; qq < kR; ++qq)
        for (int i = 0; i < nr; ++i)
          Om[size_t(qq) * nr + i] = sketch_value(RL.seed, uint64_t(lo + i), uint64_t(slot * kR + qq));
      tv[size_t(c0)] = V.m ? matmul(to_cd(V), V.m, nr, Om, kR) : std::vector<cd>();
      (void)nu_lo;
    }
    // levels 1..h: pairs (tau' in [0, 2^l), nu' of the 2^(h-l) descendants of nu at level L - l)
    for (int l = 1; l <= h; ++l) {
      const int nd = 1 << (h - l), ndp = 1 << (h - l + 1);
      std::vector<std::vector<cd>> nx(static_cast<size_t>(1 << l) * nd);
      for (int tp = 0; tp < (1 << l); ++tp)
        for (int d = 0; d < nd; ++d) {
          const int64_t nug = int64_t(nu) * nd + d;  // global index at level L - l
          const Mat &W = C[size_t(l)].fac[size_t(b)][size_t(int64_t(tp) * (int64_t(1) << (L - l)) + nug)];
          const auto &u1 = tv[size_t((tp / 2) * ndp + 2 * d)];
          const auto &u2 = tv[size_t((tp / 2) * ndp + 2 * d + 1)];
          const int r1 = int(u1.size() / size_t(kR)), r2 = int(u2.size() / size_t(kR));
          if (W.m == 0 || r1 + r2 == 0) continue;
          std::vector<cd> in(static_cast<size_t>(r1 + r2) * kR);
          for (int qq = 0; qq < kR; ++qq) {
            for (int i = 0; i < r1; ++i) in[size_t(qq) * (r1 + r2) + i] = u1[size_t(qq) * r1 + i];
            for (int i = 0; i < r2; ++i) in[size_t(qq) * (r1 + r2) + r1 + i] = u2[size_t(qq) * r2 + i];
          }
          nx[size_t(tp * nd + d)] = matmul(to_cd(W), W.m, r1 + r2, in, kR);
        }
      tv.swap(nx);
    }
    for (int tau = 0; tau < nt; ++tau) {
      const auto &Tm = tv[size_t(tau)];  // r_c x kR
      const int rc = int(Tm.size() / size_t(kR));
      const auto &gs = RL.gsel[size_t(b)][size_t(int64_t(nu) * nt + tau)];  // kR x r_r
      const int rr = int(gs.size() / size_t(kR));
      Mat &Sm = S[size_t(b)][size_t(int64_t(tau) * nn + nu)];
      Sm.m = rr;
      Sm.n = rc;
      if (rr == 0 || rc == 0) {
        Sm.v.assign(size_t(rr) * rc, cf(0, 0));
        continue;
      }
      // (T^T) S^T = G: A = T^T (kR x rc)
      std::vector<cd> A(static_cast<size_t>(kR) * rc);
      for (int c = 0; c < rc; ++c)
        for (int qq = 0; qq < kR; ++qq) A[size_t(c) * kR + qq] = Tm[size_t(qq) * rc + c];
      const std::vector<cd> St = lstsq(A, kR, rc, gs, rr);  // rc x rr
      Sm.v.resize(size_t(rr) * rc);
      for (int i = 0; i < rr; ++i)
        for (int c = 0; c < rc; ++c) Sm.v[size_t(c) * rr + i] = cf(St[size_t(i) * rc + c]);
    }
  }
  if (st) st->seconds_middle += seconds_since(tm);

  // assemble
  std::vector<Butterfly> out(static_cast<size_t>(T));
  for (int b = 0; b < T; ++b) {
    Butterfly &bf = out[size_t(b)];
    bf.hod_level = lev;
    bf.oi = tg[size_t(b)].oi;
    bf.si = tg[size_t(b)].si;
    bf.ca = tg[size_t(b)].ca;
    bf.cb = tg[size_t(b)].cb;
    bf.tau = tg[size_t(b)].tau;
    bf.L = L;
    const int64_t nl = int64_t(1) << L;
    bf.V0.resize(size_t(nl));
    for (int64_t c = 0; c < nl; ++c) bf.V0[size_t(c)] = C[0].fac[size_t(b)][size_t(c)];
    bf.W.assign(size_t(L + 1), {});
    for (int l = 1; l <= h; ++l) bf.W[size_t(l)] = C[size_t(l)].fac[size_t(b)];
    for (int l = h + 1; l <= L; ++l) {
      const int64_t na = int64_t(1) << l, nb = int64_t(1) << (L - l);
      const int j = L - l + 1;  // row-side level of the transfer factors this stage uses
      bf.W[size_t(l)].resize(size_t(na * nb));
      for (int64_t tc = 0; tc < na; ++tc)
        for (int64_t nu = 0; nu < nb; ++nu) {
          const int64_t tau = tc / 2;
          const int cc = int(tc & 1);
          // rows of the parent's row-side candidate list that belong to child tc
          const auto &sk0 = Rw[size_t(j - 1)].skel[size_t(b)][size_t(nu * (int64_t(1) << (L - j + 1)) + 2 * tau)];
          const auto &skc = Rw[size_t(j - 1)].skel[size_t(b)][size_t(nu * (int64_t(1) << (L - j + 1)) + 2 * tau + cc)];
          const int off = cc ? int(sk0.size()) : 0;
          const int mc = int(skc.size());
          std::vector<std::vector<cd>> piece(2);
          std::vector<int> pn(2);
          for (int i = 0; i < 2; ++i) {
            const int64_t nui = 2 * nu + i;
            const Mat &Vr = Rw[size_t(j)].fac[size_t(b)][size_t(nui * (int64_t(1) << (L - j)) + tau)];  // r_i x nr
            const int ri = Vr.m, nr = Vr.n;
            std::vector<cd> P(static_cast<size_t>(mc) * ri);  // rows [off, off + mc) of Vr^T
            for (int c = 0; c < ri; ++c)
              for (int r = 0; r < mc; ++r)
                P[size_t(c) * mc + r] = cd(Vr.v[size_t(off + r) * ri + c]);
            (void)nr;
            if (l == h + 1) {
              const Mat &Sm = S[size_t(b)][size_t(tau * nn + nui)];  // ri x rc
              piece[size_t(i)] = matmul(P, mc, ri, to_cd(Sm), Sm.n);
              pn[size_t(i)] = Sm.n;
            } else {
              piece[size_t(i)] = P;
              pn[size_t(i)] = ri;
            }
          }
          Mat Wm;
          Wm.m = mc;
          Wm.n = pn[0] + pn[1];
          Wm.v.reserve(size_t(Wm.m) * Wm.n);
          for (int i = 0; i < 2; ++i)
            for (const cd &v : piece[size_t(i)]) Wm.v.push_back(cf(v));
          bf.W[size_t(l)][size_t(tc * nb + nu)] = std::move(Wm);
        }
    }
    bf.B.resize(size_t(nl));
    for (int64_t a = 0; a < nl; ++a) {
      const Mat &Vr = Rw[0].fac[size_t(b)][size_t(a)];  // r x |leaf a|
      const int r = Vr.m, m = Vr.n;
      std::vector<cd> U(static_cast<size_t>(m) * r);
      for (int c = 0; c < r; ++c)
        for (int i = 0; i < m; ++i) U[size_t(c) * m + i] = cd(Vr.v[size_t(i) * r + c]);
      if (h == L) {
        const Mat &Sm = S[size_t(b)][size_t(a * nn)];  // r x rc
        bf.B[size_t(a)] = to_mat(matmul(U, m, r, to_cd(Sm), Sm.n), m, Sm.n);
      } else {
        bf.B[size_t(a)] = to_mat(U, m, r);
      }
    }
    prune_butterfly(bf);
  }
  return out;
}

// ---------------------------------------------------------------------------
// Algorithm 2 (BF_SMW) and Algorithm 1 (HODBF_invert)

namespace {

struct Ctx {
  Engine &E;
  const RbfOpts &o;
  PrecondBuild &pb;
  // final sketch widths of earlier reconstructions of the same shape and role: the next
  // one starts there instead of doubling up from k0 again
  std::map<std::tuple<int, int, int>, std::pair<int, int>> khint;
};

RowSet rows_of(const Tree &t, int lev, const std::vector<int64_t> &nodes) {
  RowSet r;
  for (int64_t v : nodes) r.push_back({t.node_lo(lev, v), t.node_hi(lev, v)});
  return r;
}

// final: the X_tau blocks a level keeps (tolerance chi); every intermediate operator of
// Algorithms 1-2 (D^{-1} B, the Schur update, the split and low-rank blocks) is
// reconstructed at chi_inner, since the inverses taken of them amplify its error
std::vector<Butterfly> rbf(Ctx &c, const LinOp &M, int lev, int L, const std::vector<Target> &tg,
                           int role, bool final = false) {
  ++c.pb.reconstructions;
  auto t0 = std::chrono::steady_clock::now();
  RbfOpts oo = c.o;
  if (!final && c.o.chi_inner > 0) oo.chi = c.o.chi_inner;
  const auto key = std::make_tuple(L, role, final ? 1 : 0);
  auto hit = c.khint.find(key);
  if (hit != c.khint.end()) {
    oo.k0_side[0] = hit->second.first;
    oo.k0_side[1] = hit->second.second;
  }
  oo.seed = mix(c.o.seed, uint64_t(c.pb.reconstructions));
  auto out = reconstruct(c.E, M, lev, L, tg, oo, &c.pb.stats);
  c.khint[key] = {c.pb.stats.last_k[0], c.pb.stats.last_k[1]};
  if (tg.size() && L >= 6)
    logf("    reconstructed %zu butterflies at level %d (%d levels) in %.2f s", tg.size(), lev, L,
         seconds_since(t0));
  return out;
}

OpP packed(Ctx &c, std::vector<Butterfly> bfs) {
  auto t0 = std::chrono::steady_clock::now();
  OpP op = c.E.butterflies(std::move(bfs));
  c.pb.stats.seconds_pack += seconds_since(t0);
  return op;
}

OpP subset_op(Ctx &c, const std::vector<Butterfly> &bfs, int ca, int cb) {
  std::vector<Butterfly> s;
  for (const auto &bf : bfs)
    if (bf.ca == ca && bf.cb == cb) s.push_back(bf);
  if (s.empty()) return nullptr;
  return packed(c, std::move(s));
}

std::vector<Target> children_targets(const std::vector<int64_t> &nodes) {
  std::vector<Target> tg;
  for (int64_t v : nodes)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) tg.push_back({2 * v + a, 2 * v + b, a, b, v});
  return tg;
}

std::vector<Butterfly> smw(Ctx &c, const std::vector<int64_t> &nodes, int lev, int Lc, OpP E11,
                           OpP E12, OpP E21, OpP E22, bool top = false);

// (I + E)^{-1} - I on the diagonal blocks (v, v) of the nodes, E given as an operator on
// those blocks whose butterfly form has Lc levels.  Splits E into its four children
// (Lc - 2 levels) and recurses; a block that cannot split is taken as one low-rank
// product B V and inverted by the Woodbury formula.
OpP inv_minus_identity(Ctx &c, const std::vector<int64_t> &nodes, int lev, int Lc, OpP E) {
  if (!E) return nullptr;
  const Tree &t = *c.E.tree;
  if (Lc - 2 < 0 || lev + 1 > t.depth) {
    std::vector<Target> tg;
    for (int64_t v : nodes) tg.push_back({v, v, 0, 0, v / 2});
    std::vector<Butterfly> lr = rbf(c, *E, lev, 0, tg, 1);
    for (Butterfly &bf : lr) {
      // E ~ B V: (I + B V)^{-1} - I = -B (I + V B)^{-1} V
      Mat &V = bf.V0[0];
      Mat &B = bf.B[0];
      const int r = V.m;
      if (r == 0 || B.n == 0) {
        B.n = 0;
        B.v.clear();
        V.m = 0;
        V.v.clear();
        continue;
      }
      std::vector<cd> K = matmul(to_cd(V), r, V.n, to_cd(B), B.n);
      for (int i = 0; i < r; ++i) K[size_t(i) * r + i] += 1.0;
      inverse_inplace(K, r);
      std::vector<cd> nb = matmul(to_cd(B), B.m, r, K, r);
      for (auto &v : nb) v = -v;
      B = to_mat(nb, B.m, r);
      ++c.pb.woodbury;
    }
    return packed(c, std::move(lr));
  }
  std::vector<Butterfly> kids = rbf(c, *E, lev + 1, Lc - 2, children_targets(nodes), 2);
  OpP C11 = subset_op(c, kids, 0, 0), C12 = subset_op(c, kids, 0, 1);
  OpP C21 = subset_op(c, kids, 1, 0), C22 = subset_op(c, kids, 1, 1);
  kids.clear();
  std::vector<Butterfly> F = smw(c, nodes, lev, Lc - 2, C11, C12, C21, C22);
  return packed(c, std::move(F));
}

// Algorithm 2 on A = I + E for every node of `nodes` (level lev), E given by its four
// child blocks (operators on (child i, child j), Lc butterfly levels each; nullptr = 0).
// Returns A^{-1} - I as four child butterflies per node with Lc levels.
std::vector<Butterfly> smw(Ctx &c, const std::vector<int64_t> &nodes, int lev, int Lc, OpP E11,
                           OpP E12, OpP E21, OpP E22, bool top) {
  const Tree &t = *c.E.tree;
  std::vector<int64_t> n1, n2;
  for (int64_t v : nodes) {
    n1.push_back(2 * v);
    n2.push_back(2 * v + 1);
  }
  // line 2: A22^{-1}
  OpP F22 = inv_minus_identity(c, n2, lev + 1, Lc, E22);
  // line 3: A11 <- A11 - A12 A22^{-1} A21 (minus I), as an operator
  OpP E11p;
  if (E12 && E21) {
    OpP mid = F22 ? plus_identity(F22) : nullptr;
    OpP coupling = mid ? chain({E21, mid, E12}) : chain({E21, E12});
    E11p = E11 ? lincomb({{1.0, E11}, {-1.0, coupling}}) : lincomb({{-1.0, coupling}});
  } else {
    E11p = E11;
  }
  // line 4: A11^{-1}
  OpP F11 = inv_minus_identity(c, n1, lev + 1, Lc, E11p);
  // line 5: A^{-1} - I as the product, reconstructed into four child butterflies
  SmwProduct prod(E12, E21, F11, F22, rows_of(t, lev + 1, n1), rows_of(t, lev + 1, n2));
  return rbf(c, prod, lev + 1, Lc, children_targets(nodes), 3, top);
}

}  // namespace

PrecondBuild invert_hodbf(Engine &E, const Kernel &ker, int min_level, int leaf_level,
                          const std::function<std::vector<Butterfly>(int)> &fwd_offdiag,
                          const RbfOpts &o) {
  const Tree &t = *E.tree;
  const int LH = t.depth;
  if (leaf_level < min_level || leaf_level > LH) fail(HODBF_E_ARG, "inverse leaf level out of range");
  PrecondBuild pb;
  pb.leaf_level = leaf_level;
  Ctx c{E, o, pb};
  auto t0 = std::chrono::steady_clock::now();
  // line 3 at the leaves of the recursion (the nodes of leaf_level): dense inverses of
  // the diagonal blocks from the kernel's entries
  const int64_t nleaf = int64_t(1) << leaf_level;
  pb.leaf_inv.resize(size_t(nleaf));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < nleaf; ++g) {
    const int32_t lo = t.node_lo(leaf_level, g), hi = t.node_hi(leaf_level, g);
    const int m = hi - lo;
    std::vector<cd> D(static_cast<size_t>(m) * m);
    for (int cc = 0; cc < m; ++cc)
      for (int r = 0; r < m; ++r) D[size_t(cc) * m + r] = ker.entry(lo + r, lo + cc);
    inverse_inplace(D, m);
    pb.leaf_inv[size_t(g)].lo = lo;
    pb.leaf_inv[size_t(g)].D = to_mat(D, m, m);
  }
  OpP leaf = E.dense_diag(pb.leaf_inv);
  pb.leaf_op = leaf;
  std::vector<OpP> built;
  logf("preconditioner: %lld dense inverses at level %d, %.2f s", (long long)nleaf, leaf_level,
       seconds_since(t0));
  for (int l = leaf_level - 1; l >= min_level; --l) {
    auto tl = std::chrono::steady_clock::now();
    const int Lb = LH - l - 1;
    std::vector<int64_t> nodes(static_cast<size_t>(int64_t(1) << l));
    for (size_t i = 0; i < nodes.size(); ++i) nodes[i] = int64_t(i);
    // line 7: B_tau_i <- D_tau_i^{-1} B_tau_i for both children of every node
    OpP O = packed(c, fwd_offdiag(l));
    OpP Dinv = mult_inverse(E, leaf, built);
    OpP M7 = chain({O, Dinv});
    std::vector<Target> tg;
    for (int64_t v : nodes) {
      tg.push_back({2 * v, 2 * v + 1, 0, 1, v});
      tg.push_back({2 * v + 1, 2 * v, 1, 0, v});
    }
    std::vector<Butterfly> Bp = rbf(c, *M7, l + 1, Lb, tg, 0);
    O.reset();
    M7.reset();
    OpP E12 = subset_op(c, Bp, 0, 1), E21 = subset_op(c, Bp, 1, 0);
    Bp.clear();
    // line 8: D_tau^{-1} = BF_SMW([I, B1; B2, I]) diag(D1^{-1}, D2^{-1})
    std::vector<Butterfly> X = smw(c, nodes, l, Lb, nullptr, E12, E21, nullptr, true);
    built.push_back(packed(c, X));
    pb.levels.push_back(std::move(X));
    pb.ops.push_back(built.back());
    logf("preconditioner level %d: %lld nodes, %.2f s (%.2f s so far), %lld reconstructions, "
         "%lld sketch columns (%lld redone levels), largest rank %d; seconds so far: products "
         "%.1f, IDs %.1f, middle %.1f, packing %.1f", l, (long long)nodes.size(), seconds_since(tl),
         seconds_since(t0), (long long)pb.reconstructions, (long long)pb.stats.sketch_cols,
         (long long)pb.stats.redone, pb.stats.max_rank, pb.stats.seconds_apply, pb.stats.seconds_id,
         pb.stats.seconds_middle, pb.stats.seconds_pack);
  }
  return pb;
}

}  // namespace hodbf
