// Host construction of nested-ID butterflies (Section III-A, eqs. (ID), (nested_basis),
// (butterfly_mat)) with sampled rows, level-synchronous and OpenMP-parallel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace hodbf {

namespace {

uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct ZSource final : EntrySource {
  const Kernel *k;
  explicit ZSource(const Kernel *kk) : k(kk) { tree = kk->tree; }
  void fill(const int32_t *rows, int nr, const int32_t *cols, int nc, cd *out) const override {
    for (int c = 0; c < nc; ++c)
      for (int r = 0; r < nr; ++r) out[size_t(c) * nr + r] = k->entry(rows[r], cols[c]);
  }
};

// Rows of [r0, r1) used for one ID of M = A(rows, cols) and their weights.
// Few rows: all of them (the ID is then exact in the sense of eq. (ID)).
// Otherwise: every row inside the columns' bounding box grown by two voxels (the
// near field that dominates weakly admissible blocks), plus mult * (2*nc+16) uniform
// random rows from the rest, weighted by sqrt(remaining / drawn) so that Frobenius
// norms of the sample estimate those of the full block and the chi test keeps its
// meaning.  rest receives the far rows that were not drawn (empty when every row is
// used), from which the ID is then checked.
void pick_rows(const Tree &t, int32_t r0, int32_t r1, const std::vector<int32_t> &cols,
               uint64_t seed, int mult, std::vector<int32_t> &rows, std::vector<double> &wt,
               std::vector<int32_t> &rest) {
  const int32_t m = r1 - r0;
  const int nc = int(cols.size());
  rows.clear();
  wt.clear();
  rest.clear();
  if (m <= 2 * nc + 48) {
    rows.resize(m);
    std::iota(rows.begin(), rows.end(), r0);
    wt.assign(m, 1.0);
    return;
  }
  int lo[3] = {1 << 20, 1 << 20, 1 << 20}, hi[3] = {-(1 << 20), -(1 << 20), -(1 << 20)};
  for (int32_t c : cols) {
    const int v[3] = {t.cx[c], t.cy[c], t.cz[c]};
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], v[a] - 2);
      hi[a] = std::max(hi[a], v[a] + 2);
    }
  }
  std::vector<int32_t> far;
  far.reserve(m);
  for (int32_t r = r0; r < r1; ++r) {
    const int v[3] = {t.cx[r], t.cy[r], t.cz[r]};
    const bool near = v[0] >= lo[0] && v[0] <= hi[0] && v[1] >= lo[1] && v[1] <= hi[1] &&
                      v[2] >= lo[2] && v[2] <= hi[2];
    if (near) {
      rows.push_back(r);
      wt.push_back(1.0);
    } else {
      far.push_back(r);
    }
  }
  const int64_t want = std::min<int64_t>(far.size(), int64_t(mult) * (2 * int64_t(nc) + 16));
  if (want == int64_t(far.size())) {
    for (int32_t r : far) {
      rows.push_back(r);
      wt.push_back(1.0);
    }
    return;
  }
  uint64_t s = seed;
  for (int64_t i = 0; i < want; ++i) {  // partial Fisher-Yates
    const int64_t j = i + int64_t(splitmix(s) % uint64_t(far.size() - i));
    std::swap(far[i], far[j]);
  }
  std::sort(far.begin(), far.begin() + want);
  const double w = std::sqrt(double(far.size()) / double(want));
  for (int64_t i = 0; i < want; ++i) {
    rows.push_back(far[i]);
    wt.push_back(w);
  }
  rest.assign(far.begin() + want, far.end());
}

// Squared Frobenius norm of A(rows, cols) - A(rows, cols(J)) V over up to 32 rows drawn
// from `rest`, scaled to all of `rest` (V: r x nc column-major, V(:, J) = I).
double check_rows_residual2(const EntrySource &src, const std::vector<int32_t> &rest,
                            const std::vector<int32_t> &cols, const std::vector<int> &J,
                            const std::vector<cd> &V, int rk, uint64_t seed) {
  const int nc = int(cols.size());
  std::vector<int32_t> pool(rest);
  const int nv = int(std::min<size_t>(pool.size(), 32));
  uint64_t s = seed;
  for (int i = 0; i < nv; ++i) {
    const size_t j = size_t(i) + size_t(splitmix(s) % uint64_t(pool.size() - size_t(i)));
    std::swap(pool[size_t(i)], pool[j]);
  }
  std::vector<cd> Mv(size_t(nv) * nc);
  src.fill(pool.data(), nv, cols.data(), nc, Mv.data());
  double r2 = 0;
  for (int i = 0; i < nv; ++i)
    for (int c = 0; c < nc; ++c) {
      cd e = Mv[size_t(c) * nv + i];
      for (int k = 0; k < rk; ++k) e -= Mv[size_t(J[k]) * nv + i] * V[size_t(c) * rk + k];
      r2 += std::norm(e);
    }
  return r2 * double(rest.size()) / double(std::max(nv, 1));
}

uint64_t job_seed(uint64_t seed, int64_t bf, int l, int64_t a, int64_t b) {
  uint64_t s = seed ^ 0x5DEECE66Dull;
  s ^= splitmix(s) + uint64_t(bf) * 0x100000001B3ull;
  s ^= splitmix(s) + uint64_t(l) * 0x9E3779B1ull;
  s ^= splitmix(s) + uint64_t(a) * 0xC2B2AE35ull;
  s ^= splitmix(s) + uint64_t(b) * 0x27D4EB2Full;
  return splitmix(s);
}

}  // namespace

// Build every butterfly in bfs (hod_level, oi, si, L preset) level by level: all IDs
// of butterfly level l are independent once level l-1 is known.
void build_butterflies(const EntrySource &src, const Tree &t, std::vector<Butterfly> &bfs,
                       double chi, uint64_t seed, int64_t *id_count) {
  int Lmax = -1;
  for (auto &bf : bfs) Lmax = std::max(Lmax, bf.L);
  std::vector<std::vector<std::vector<int32_t>>> skel(bfs.size()), nskel(bfs.size());
  struct Job {
    int64_t bf, a, b;
    double cost;
  };
  int64_t ids = 0, redo = 0;
  for (int l = 0; l <= Lmax; ++l) {
    std::vector<Job> jobs;
    for (size_t k = 0; k < bfs.size(); ++k) {
      Butterfly &bf = bfs[k];
      if (bf.L < l) continue;
      const int64_t na = int64_t(1) << l, nb = int64_t(1) << (bf.L - l);
      if (l == 0) bf.V0.assign(static_cast<size_t>(nb), Mat{});
      else {
        if (int(bf.W.size()) <= bf.L) bf.W.resize(bf.L + 1);
        bf.W[l].assign(static_cast<size_t>(na * nb), Mat{});
      }
      nskel[k].assign(static_cast<size_t>(na * nb), {});
      for (int64_t a = 0; a < na; ++a)
        for (int64_t b = 0; b < nb; ++b) {
          const int lev = bf.hod_level + l;
          const int64_t rows = t.node_hi(lev, bf.oi * na + a) - t.node_lo(lev, bf.oi * na + a);
          double nc;
          if (l == 0) {
            const int leaf = bf.hod_level + bf.L;
            nc = t.node_hi(leaf, bf.si * nb + b) - t.node_lo(leaf, bf.si * nb + b);
          } else {
            nc = double(skel[k][size_t((a / 2) * 2 * nb + 2 * b)].size() +
                        skel[k][size_t((a / 2) * 2 * nb + 2 * b + 1)].size());
          }
          jobs.push_back({int64_t(k), a, b, std::min<double>(rows, 2 * nc + 64) * nc * nc});
        }
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job &x, const Job &y) { return x.cost > y.cost; });
    ids += int64_t(jobs.size());
#pragma omp parallel
    {
      std::vector<int32_t> cols, rows, rest;
      std::vector<double> wt;
      std::vector<cd> M, V;
      std::vector<int> J;
#pragma omp for schedule(dynamic, 1)
      for (int64_t q = 0; q < int64_t(jobs.size()); ++q) {
        const Job &jb = jobs[q];
        Butterfly &bf = bfs[jb.bf];
        const int64_t na = int64_t(1) << l, nb = int64_t(1) << (bf.L - l);
        const int lev = bf.hod_level + l;
        const int64_t tau = bf.oi * na + jb.a;
        const int32_t r0 = t.node_lo(lev, tau), r1 = t.node_hi(lev, tau);
        cols.clear();
        if (l == 0) {
          const int leaf = bf.hod_level + bf.L;
          const int64_t nu = bf.si * nb + jb.b;
          for (int32_t c = t.node_lo(leaf, nu); c < t.node_hi(leaf, nu); ++c) cols.push_back(c);
        } else {
          const auto &s1 = skel[jb.bf][size_t((jb.a / 2) * 2 * nb + 2 * jb.b)];
          const auto &s2 = skel[jb.bf][size_t((jb.a / 2) * 2 * nb + 2 * jb.b + 1)];
          cols.insert(cols.end(), s1.begin(), s1.end());
          cols.insert(cols.end(), s2.begin(), s2.end());
        }
        const int nc = int(cols.size());
        Mat out;
        out.n = nc;
        std::vector<int32_t> sk;
        if (nc > 0) {
          // the ID of the sampled rows is checked on rows it did not see: if the residual
          // estimated from them exceeds 2 chi ||M||_F (the sampled rows' own residual is
          // just under chi ||M||_F, and 32 rows estimate the rest only roughly), the random
          // sample doubles and the ID is redone (at most three times)
          const uint64_t js = job_seed(seed, jb.bf, l, jb.a, jb.b);
          int rk = 0;
          for (int mult = 1;; mult *= 2) {
            pick_rows(*src.tree, r0, r1, cols, js, mult, rows, wt, rest);
            const int nr = int(rows.size());
            M.resize(size_t(nr) * nc);
            src.fill(rows.data(), nr, cols.data(), nc, M.data());
            double norm2 = 0;
            for (int c = 0; c < nc; ++c)
              for (int r = 0; r < nr; ++r) {
                M[size_t(c) * nr + r] *= wt[r];
                norm2 += std::norm(M[size_t(c) * nr + r]);
              }
            rk = id_cpqr(M.data(), nr, nc, chi, J, V);
            if (rest.empty() || mult >= 8) break;
            const double res2 = check_rows_residual2(src, rest, cols, J, V, rk, js ^ 0xC0FFEEull);
            if (res2 <= 4 * chi * chi * norm2) break;
#pragma omp atomic
            ++redo;
          }
          out.m = rk;
          out.v.assign(V.begin(), V.end());
          sk.resize(rk);
          for (int i = 0; i < rk; ++i) sk[i] = cols[J[i]];
        }
        if (l == 0) bf.V0[size_t(jb.b)] = std::move(out);
        else bf.W[l][size_t(jb.a * nb + jb.b)] = std::move(out);
        nskel[jb.bf][size_t(jb.a * nb + jb.b)] = std::move(sk);
      }
    }
    for (size_t k = 0; k < bfs.size(); ++k)
      if (bfs[k].L >= l) skel[k].swap(nskel[k]);
    if (jobs.size() >= 100000) logf("  butterfly level %d: %zu IDs done", l, jobs.size());
  }
  for (size_t k = 0; k < bfs.size(); ++k) {
    Butterfly &bf = bfs[k];
    const int64_t na = int64_t(1) << bf.L;
    bf.bskel.assign(static_cast<size_t>(na), {});
    for (int64_t a = 0; a < na; ++a) bf.bskel[size_t(a)] = skel[k][size_t(a)];
  }
  if (id_count) *id_count += ids;
  if (redo) logf("  row sampling: %lld IDs redone with a doubled sample", (long long)redo);
}

void validate_params(const hodbf_build_params &p) {
  if (p.nx <= 0 || p.ny <= 0 || p.nz <= 0) fail(HODBF_E_ARG, "grid sides must be positive");
  if (int64_t(p.nx) * p.ny * p.nz > (int64_t(1) << 30)) fail(HODBF_E_ARG, "grid too large");
  if (std::max({p.nx, p.ny, p.nz}) > 30000) fail(HODBF_E_ARG, "grid side too large");
  if (!(p.h > 0) || !std::isfinite(p.h)) fail(HODBF_E_ARG, "h must be positive");
  if (!(p.k0 > 0) || !std::isfinite(p.k0)) fail(HODBF_E_ARG, "k0 must be positive");
  if (!(p.tol_con > 0 && p.tol_con < 1)) fail(HODBF_E_ARG, "tol_con must lie in (0, 1)");
  if (p.precond_prec != HODBF_P_NONE && !(p.tol_fact > 0 && p.tol_fact < 1))
    fail(HODBF_E_ARG, "tol_fact must lie in (0, 1)");
  if (p.leaf_size < 1 || p.leaf_size > 64) fail(HODBF_E_ARG, "leaf_size must be 1..64");
  if (p.precond_prec < 0 || p.precond_prec > 7)
    fail(HODBF_E_ARG, "unknown precond_prec");
  if (p.precond_min_level < 0) fail(HODBF_E_ARG, "precond_min_level must be >= 0");
  if (p.precond_dense_levels < 0) fail(HODBF_E_ARG, "precond_dense_levels must be >= 0");
  if (!p.eps_r) fail(HODBF_E_ARG, "eps_r is NULL");
  const int64_t n = int64_t(p.nx) * p.ny * p.nz;
  for (int64_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(p.eps_r[i])) fail(HODBF_E_ARG, "eps_r holds a non-finite value");
  for (int64_t i = 0; i < n; ++i)
    if (p.eps_r[2 * i] == 0.0 && p.eps_r[2 * i + 1] == 0.0) fail(HODBF_E_ARG, "eps_r = 0");
}

FwdPlan build_forward_plan(const hodbf_build_params &p) {
  validate_params(p);
  FwdPlan fp;
  fp.tree = build_tree(p.nx, p.ny, p.nz, p.leaf_size);
  const int64_t n = fp.tree.n;
  std::vector<cd> eps(n);
  for (int64_t i = 0; i < n; ++i) eps[i] = cd(p.eps_r[2 * i], p.eps_r[2 * i + 1]);
  fp.ker = make_kernel(fp.tree, eps, p.h, p.k0);
  const int LH = fp.tree.depth;
  for (int l = 1; l <= LH; ++l)
    for (int64_t i = 0; i < (int64_t(1) << l); ++i) {
      Butterfly bf;
      bf.hod_level = l;
      bf.oi = i;
      bf.si = i ^ 1;
      bf.L = LH - l;
      fp.bfs.push_back(std::move(bf));
    }
  ZSource src(&fp.ker);
  build_butterflies(src, fp.tree, fp.bfs, p.tol_con, p.seed, &fp.id_count);
  int mr = 0;
  for (auto &bf : fp.bfs) {
    for (auto &v : bf.V0) mr = std::max(mr, v.m);
    for (int l = 1; l <= bf.L; ++l)
      for (auto &w : bf.W[l]) mr = std::max(mr, w.m);
  }
  fp.max_rank = mr;
  return fp;
}

}  // namespace hodbf
