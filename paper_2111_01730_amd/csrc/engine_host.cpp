// Host engine of the preconditioner construction: multi-vectors in complex FP64 on the
// CPU, butterflies and dense blocks applied by plain loops.  It runs the same Algorithm
// 1 / Algorithm 2 code as the device engine, for small problems and verification.
#include <algorithm>
#include <cmath>
#include <limits>

#include "construct.h"
#include "pack_sink.h"

namespace hodbf {

namespace {

struct HostMv final : Mv {
  std::vector<cd> d;  // element (i, q) at i * R + q
};

const HostMv &hv(const Mv &m) { return static_cast<const HostMv &>(m); }
HostMv &hv(Mv &m) { return static_cast<HostMv &>(m); }

// out(m x R, row-major) (+)= F (m x n, column-major; trans: F^T, F being n x m) times
// x (n x R, row-major)
void gemm_rows(const Mat &F, bool trans, const cd *x, int R, cd *out, bool accumulate) {
  const int m = trans ? F.n : F.m, n = trans ? F.m : F.n;
  if (!accumulate) std::fill(out, out + size_t(m) * R, cd(0, 0));
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < m; ++i) {
      const cd a = trans ? cd(F.v[size_t(i) * F.m + k]) : cd(F.v[size_t(k) * F.m + i]);
      if (a == cd(0, 0)) continue;
      const cd *xr = x + size_t(k) * R;
      cd *o = out + size_t(i) * R;
      for (int q = 0; q < R; ++q) o[q] += a * xr[q];
    }
}

class HostBf final : public LinOp {
 public:
  HostBf(const Tree *t, std::vector<Butterfly> bfs) : t_(t), bfs_(std::move(bfs)) {}
  void apply(Engine &, bool trans, const Mv &x, Mv &y) const override {
    const auto &X = hv(x).d;
    auto &Y = hv(y).d;
    const int R = x.R;
    std::fill(Y.begin(), Y.end(), cd(0, 0));
    // butterflies that write the same rows run one after another; others in parallel
    std::vector<std::vector<size_t>> groups;
    {
      std::vector<std::pair<int64_t, size_t>> key;
      for (size_t k = 0; k < bfs_.size(); ++k)
        key.push_back({trans ? bfs_[k].si : bfs_[k].oi, k});
      std::sort(key.begin(), key.end());
      for (size_t i = 0; i < key.size(); ++i) {
        if (i == 0 || key[i].first != key[i - 1].first) groups.emplace_back();
        groups.back().push_back(key[i].second);
      }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < int64_t(groups.size()); ++g)
      for (size_t k : groups[size_t(g)]) one(bfs_[k], trans, X.data(), R, Y.data());
  }

 private:
  void one(const Butterfly &bf, bool trans, const cd *x, int R, cd *y) const {
    const Tree &t = *t_;
    const int L = bf.L, ll = bf.hod_level + L;
    const int64_t nl = int64_t(1) << L;
    auto rng = [&](int64_t top, int64_t i) { return std::make_pair(t.node_lo(ll, (top << L) + i), t.node_hi(ll, (top << L) + i)); };
    if (!trans) {
      std::vector<std::vector<cd>> tv(static_cast<size_t>(nl));
      for (int64_t b = 0; b < nl; ++b) {
        const Mat &V = bf.V0[size_t(b)];
        tv[size_t(b)].assign(size_t(V.m) * R, cd(0, 0));
        if (V.m) gemm_rows(V, false, x + size_t(rng(bf.si, b).first) * R, R, tv[size_t(b)].data(), false);
      }
      for (int l = 1; l <= L; ++l) {
        const int64_t na = int64_t(1) << l, nb = int64_t(1) << (L - l);
        std::vector<std::vector<cd>> nx(static_cast<size_t>(na * nb));
        for (int64_t a = 0; a < na; ++a)
          for (int64_t b = 0; b < nb; ++b) {
            const Mat &W = bf.W[size_t(l)][size_t(a * nb + b)];
            const auto &u1 = tv[size_t((a / 2) * 2 * nb + 2 * b)];
            const auto &u2 = tv[size_t((a / 2) * 2 * nb + 2 * b + 1)];
            std::vector<cd> in(u1);
            in.insert(in.end(), u2.begin(), u2.end());
            auto &o = nx[size_t(a * nb + b)];
            o.assign(size_t(W.m) * R, cd(0, 0));
            if (W.m && W.n) gemm_rows(W, false, in.data(), R, o.data(), false);
          }
        tv.swap(nx);
      }
      for (int64_t a = 0; a < nl; ++a) {
        const Mat &B = bf.B[size_t(a)];
        if (B.n) gemm_rows(B, false, tv[size_t(a)].data(), R, y + size_t(rng(bf.oi, a).first) * R, true);
      }
      return;
    }
    // transposed: the stages in reverse, each factor transposed
    std::vector<std::vector<cd>> tv(static_cast<size_t>(nl));
    for (int64_t a = 0; a < nl; ++a) {
      const Mat &B = bf.B[size_t(a)];
      tv[size_t(a)].assign(size_t(B.n) * R, cd(0, 0));
      if (B.n) gemm_rows(B, true, x + size_t(rng(bf.oi, a).first) * R, R, tv[size_t(a)].data(), false);
    }
    for (int l = L; l >= 1; --l) {
      const int64_t na = int64_t(1) << l, nb = int64_t(1) << (L - l);
      // outputs of stage l - 1: (a', b') with a' < na / 2, b' < 2 nb
      std::vector<std::vector<cd>> pv(static_cast<size_t>((na / 2) * (2 * nb)));
      for (int64_t ap = 0; ap < na / 2; ++ap)
        for (int64_t b = 0; b < nb; ++b) {
          // sizes of the two stage l - 1 outputs this input segment holds
          const int r1 = l - 1 == 0 ? bf.V0[size_t(2 * b)].m
                                    : bf.W[size_t(l - 1)][size_t(ap * (2 * nb) + 2 * b)].m;
          const int r2 = l - 1 == 0 ? bf.V0[size_t(2 * b + 1)].m
                                    : bf.W[size_t(l - 1)][size_t(ap * (2 * nb) + 2 * b + 1)].m;
          const int ntot = r1 + r2;
          std::vector<cd> acc(static_cast<size_t>(ntot) * R, cd(0, 0));
          for (int c = 0; c < 2; ++c) {
            const Mat &W = bf.W[size_t(l)][size_t((2 * ap + c) * nb + b)];
            if (W.m && W.n == ntot && ntot)
              gemm_rows(W, true, tv[size_t((2 * ap + c) * nb + b)].data(), R, acc.data(), true);
          }
          pv[size_t(ap * 2 * nb + 2 * b)].assign(acc.begin(), acc.begin() + size_t(r1) * R);
          pv[size_t(ap * 2 * nb + 2 * b + 1)].assign(acc.begin() + size_t(r1) * R, acc.end());
        }
      tv.swap(pv);
    }
    for (int64_t b = 0; b < nl; ++b) {
      const Mat &V = bf.V0[size_t(b)];
      if (V.m) gemm_rows(V, true, tv[size_t(b)].data(), R, y + size_t(rng(bf.si, b).first) * R, true);
    }
  }

  const Tree *t_;
  std::vector<Butterfly> bfs_;
};

class HostDense final : public LinOp {
 public:
  explicit HostDense(std::vector<DenseDiag> b) : b_(std::move(b)) {}
  void apply(Engine &, bool trans, const Mv &x, Mv &y) const override {
    const auto &X = hv(x).d;
    auto &Y = hv(y).d;
    const int R = x.R;
    std::fill(Y.begin(), Y.end(), cd(0, 0));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < int64_t(b_.size()); ++i) {
      const DenseDiag &d = b_[size_t(i)];
      gemm_rows(d.D, trans, X.data() + size_t(d.lo) * R, R, Y.data() + size_t(d.lo) * R, false);
    }
  }

 private:
  std::vector<DenseDiag> b_;
};

// The packed grouped-GEMM programs of the device path, run by a host interpreter with
// the kernels' semantics: every tile sums its pairs (factor column-major at f_off with
// lda, times input rows of X or T) and scatters its rows through the row map into T or
// OUT (beta 0 stores, beta 1 adds).  T starts as NaN, so a read of a row no earlier
// launch wrote poisons the result.
class HostProgOp final : public LinOp {
 public:
  PackSink fwd, trans;
  std::vector<cd> arena;
  void apply(Engine &E, bool tr, const Mv &x, Mv &y) const override {
    const PackSink &pk = tr ? trans : fwd;
    const int R = x.R;
    const auto &X = hv(x).d;
    auto &Y = hv(y).d;
    std::fill(Y.begin(), Y.end(), cd(0, 0));
    std::vector<cd> T(size_t(std::max<int64_t>(pk.t_rows, 1)) * R,
                      cd(std::numeric_limits<double>::quiet_NaN(), 0.0));
    std::vector<cd> acc;
    for (const Launch &ln : pk.launches)
      for (int64_t s = ln.s0; s < ln.s0 + ln.ns; ++s) {
        const Seg &sg = pk.segs[size_t(s)];
        acc.assign(size_t(sg.m) * R, cd(0, 0));
        for (int32_t p = sg.p0; p < sg.p1; ++p) {
          const Pair &pr = pk.pairs[size_t(p)];
          const cd *in = (pr.in_buf ? T.data() : X.data()) + size_t(pr.in_row) * R;
          for (int k = 0; k < pr.n; ++k)
            for (int i = 0; i < sg.m; ++i) {
              const cd a = arena[size_t(pr.f_off + int64_t(k) * pr.lda + i)] * double(pr.scale);
              for (int q = 0; q < R; ++q) acc[size_t(i) * R + q] += a * in[size_t(k) * R + q];
            }
        }
        cd *dst = ln.out ? Y.data() : T.data();
        for (int i = 0; i < sg.m; ++i) {
          int32_t base = 0;
          for (int32_t e = sg.map0; e < sg.map1; ++e)
            if (pk.rowmap[size_t(e)].start <= i) base = pk.rowmap[size_t(e)].out_row - pk.rowmap[size_t(e)].start;
          cd *o = dst + size_t(base + i) * R;
          for (int q = 0; q < R; ++q) o[q] = ln.beta ? o[q] + acc[size_t(i) * R + q] : acc[size_t(i) * R + q];
        }
      }
    (void)E;
  }
};

class HostEngine final : public Engine {
 public:
  HostEngine(const Tree *t, int mc, bool programs) : mc_(mc), programs_(programs) { tree = t; }
  int max_cols() const override { return mc_; }
  MvP make(int R) override {
    auto m = std::make_shared<HostMv>();
    m->R = R;
    m->d.assign(size_t(n()) * R, cd(0, 0));
    return m;
  }
  void zero(Mv &y) override { std::fill(hv(y).d.begin(), hv(y).d.end(), cd(0, 0)); }
  void copy(const Mv &x, Mv &y) override { hv(y).d = hv(x).d; }
  void axpy(cd a, const Mv &x, Mv &y) override {
    const auto &X = hv(x).d;
    auto &Y = hv(y).d;
    for (size_t i = 0; i < Y.size(); ++i) Y[i] += a * X[i];
  }
  void keep_rows(const RowSet &rows, Mv &y) override {
    auto &Y = hv(y).d;
    std::vector<char> keep(static_cast<size_t>(n()), 0);
    for (auto [lo, hi] : rows)
      for (int32_t r = lo; r < hi; ++r) keep[size_t(r)] = 1;
    for (int64_t r = 0; r < n(); ++r)
      if (!keep[size_t(r)]) std::fill(Y.begin() + r * y.R, Y.begin() + (r + 1) * y.R, cd(0, 0));
  }
  void fill_sketch(Mv &x, const std::vector<int32_t> &slot_of_row, int64_t col0, int k,
                   uint64_t seed) override {
    auto &X = hv(x).d;
    const int R = x.R;
    std::fill(X.begin(), X.end(), cd(0, 0));
    for (int64_t r = 0; r < n(); ++r) {
      const int32_t s = slot_of_row[size_t(r)];
      if (s < 0) continue;
      for (int i = 0; i < k; ++i) {
        const int64_t g = int64_t(s) * k + i;
        if (g < col0 || g >= col0 + R) continue;
        X[size_t(r) * R + size_t(g - col0)] = sketch_value(seed, uint64_t(r), uint64_t(g));
      }
    }
  }
  void fill_unit(Mv &x, const std::vector<int32_t> &col_of_row) override {
    auto &X = hv(x).d;
    std::fill(X.begin(), X.end(), cd(0, 0));
    for (int64_t r = 0; r < n(); ++r) {
      const int32_t c = col_of_row[size_t(r)];
      if (c >= 0 && c < x.R) X[size_t(r) * x.R + size_t(c)] = 1.0;
    }
  }
  void gather(const Mv &y, const std::vector<Gather> &req, int k, std::vector<cd> &out) override {
    const auto &Y = hv(y).d;
    out.clear();
    for (const Gather &g : req)
      for (int32_t r : g.rows)
        for (int i = 0; i < k; ++i) out.push_back(Y[size_t(r) * y.R + size_t(g.q0 + i)]);
  }
  OpP butterflies(std::vector<Butterfly> bfs) override {
    if (!programs_) return std::make_shared<HostBf>(tree, std::move(bfs));
    auto op = std::make_shared<HostProgOp>();
    for (Butterfly &bf : bfs) prune_butterfly(bf);
    std::vector<const Butterfly *> ptrs;
    for (const Butterfly &bf : bfs) ptrs.push_back(&bf);
    std::vector<BlockRec> table;
    for (int dir = 0; dir < 2; ++dir) {
      PackSink &pk = dir == 0 ? op->fwd : op->trans;
      pk.table = &table;
      pk.put_host = [&](const Mat &f, float *scale) { return put(op->arena, f, scale); };
      if (dir == 0)
        pack_group(pk, *tree, ptrs, false, 0, [](const Butterfly &, int64_t *md) {
          md[0] = md[1] = md[2] = md[3] = 0;
        });
      else
        pack_group_t(pk, *tree, ptrs);
      check_program(pk, n(), -1);
    }
    for (int dir = 0; dir < 2; ++dir) {
      PackSink &pk = dir == 0 ? op->fwd : op->trans;
      retile(pk, kRetileBelow, kTileRows / 2);
      check_program(pk, n(), int64_t(op->arena.size()));
      pk.table = nullptr;
      pk.put_host = nullptr;
    }
    return op;
  }
  OpP dense_diag(std::vector<DenseDiag> blocks) override { return std::make_shared<HostDense>(std::move(blocks)); }

 private:
  static int64_t put(std::vector<cd> &arena, const Mat &f, float *scale) {
    *scale = 1.0f;
    const int64_t off = (int64_t(arena.size()) + 15) & ~int64_t(15);
    arena.resize(size_t(off + int64_t(f.m) * f.n), cd(0, 0));
    for (size_t e = 0; e < f.v.size(); ++e) arena[size_t(off) + e] = cd(f.v[e]);
    return off;
  }
  int mc_;
  bool programs_;
};

}  // namespace

std::unique_ptr<Engine> make_host_engine(const Tree *t, int max_cols, bool programs) {
  return std::make_unique<HostEngine>(t, max_cols, programs);
}

}  // namespace hodbf
