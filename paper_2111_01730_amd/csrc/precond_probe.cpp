// Host-only run of the preconditioner construction (Algorithm 1 with Algorithm 2 and
// randomized reconstruction, complex FP64 on the CPU) for verification without a GPU,
// and helpers shared with the device construction: the forward operator's off-diagonal
// butterflies with explicit outer factors, and the block-table export.
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "construct.h"
#include "precond_host.h"

namespace hodbf {

std::vector<Butterfly> forward_offdiag_explicit(const Tree &t, const std::vector<Butterfly> &plan,
                                               const Kernel &ker, int l) {
  const int LH = t.depth;
  std::vector<Butterfly> out;
  for (const Butterfly &src : plan) {
    if (src.hod_level != l + 1) continue;
    Butterfly bf;
    bf.hod_level = src.hod_level;
    bf.oi = src.oi;
    bf.si = src.si;
    bf.ca = int(src.oi & 1);
    bf.cb = int(src.si & 1);
    bf.tau = src.oi >> 1;
    bf.L = src.L;
    bf.V0 = src.V0;
    bf.W = src.W;
    out.push_back(std::move(bf));
  }
  // outer factors B^L = Z(tau_a, sbar_a) from the kernel entries
  std::vector<std::pair<size_t, int64_t>> jobs;
  size_t k = 0;
  for (const Butterfly &src : plan) {
    if (src.hod_level != l + 1) continue;
    out[k].B.resize(size_t(int64_t(1) << src.L));
    for (int64_t a = 0; a < (int64_t(1) << src.L); ++a) jobs.push_back({k, a});
    ++k;
  }
  std::vector<const Butterfly *> srcs;
  for (const Butterfly &src : plan)
    if (src.hod_level == l + 1) srcs.push_back(&src);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < int64_t(jobs.size()); ++q) {
    const auto [bi, a] = jobs[size_t(q)];
    const Butterfly &src = *srcs[bi];
    const int64_t leaf = (src.oi << src.L) + a;
    const int32_t lo = t.node_lo(LH, leaf), hi = t.node_hi(LH, leaf);
    const auto &sk = src.bskel[size_t(a)];
    Mat &B = out[bi].B[size_t(a)];
    B.m = hi - lo;
    B.n = int(sk.size());
    B.v.resize(size_t(B.m) * B.n);
    for (int c = 0; c < B.n; ++c)
      for (int r = 0; r < B.m; ++r) B.v[size_t(c) * B.m + r] = cf(ker.entry(lo + r, sk[size_t(c)]));
  }
  return out;
}

void export_precond_build(const PrecondBuild &pb, std::vector<BlockRec> &table,
                          std::vector<cd> &vals) {
  table.clear();
  vals.clear();
  auto put = [&](const Mat &f) {
    const int64_t off = int64_t(vals.size());
    for (const cf &v : f.v) vals.push_back(cd(v));
    return off;
  };
  for (size_t g = 0; g < pb.leaf_inv.size(); ++g) {
    const Mat &D = pb.leaf_inv[g].D;
    table.push_back({0, pb.leaf_level, int64_t(g), 0, 0, 0, 0, 0, D.m, D.n, put(D), D.m});
  }
  for (const auto &lvl : pb.levels)
    for (const Butterfly &bf : lvl) {
      const int64_t l = bf.hod_level - 1;
      for (int64_t b = 0; b < int64_t(bf.V0.size()); ++b) {
        const Mat &f = bf.V0[size_t(b)];
        if (f.m) table.push_back({1, l, bf.tau, bf.ca, bf.cb, 0, 0, b, f.m, f.n, put(f), f.m});
      }
      for (int s = 1; s <= bf.L; ++s) {
        const int64_t nb = int64_t(1) << (bf.L - s);
        for (int64_t e = 0; e < int64_t(bf.W[size_t(s)].size()); ++e) {
          const Mat &f = bf.W[size_t(s)][size_t(e)];
          if (f.m && f.n)
            table.push_back({2, l, bf.tau, bf.ca, bf.cb, s, e / nb, e % nb, f.m, f.n, put(f), f.m});
        }
      }
      for (int64_t a = 0; a < int64_t(bf.B.size()); ++a) {
        const Mat &f = bf.B[size_t(a)];
        if (f.n) table.push_back({3, l, bf.tau, bf.ca, bf.cb, bf.L, a, 0, f.m, f.n, put(f), f.m});
      }
    }
}

}  // namespace hodbf

using namespace hodbf;

namespace {
std::mutex g_pp_mu;
std::vector<double> g_pp_key;
std::vector<int32_t> g_pp_perm;
std::vector<BlockRec> g_pp_table;
std::vector<cd> g_pp_vals;
std::vector<int64_t> g_pp_stats;

void pp_export(const void *src, size_t n, void *buf, size_t *bytes) {
  if (!buf) {
    *bytes = n;
    return;
  }
  if (*bytes < n) fail(HODBF_E_ARG, "export buffer too small");
  if (n) std::memcpy(buf, src, n);
  *bytes = n;
}
}  // namespace

extern "C" hodbf_status hodbf_precond_probe(const hodbf_build_params *params, int32_t which,
                                            void *buf, size_t *bytes) {
  return hodbf_guarded([&] {
    if (!params || !bytes) fail(HODBF_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_pp_mu);
    const int64_t n = int64_t(params->nx) * params->ny * params->nz;
    if (n > 65536) fail(HODBF_E_ARG, "the host construction is for small problems (N <= 65536)");
    const bool programs = which >= 16;
    if (programs) which -= 16;
    std::vector<double> key = {double(programs), double(params->nx), double(params->ny), double(params->nz),
                               params->h, params->k0, params->tol_con, params->tol_fact,
                               double(params->leaf_size), double(params->seed),
                               double(params->precond_min_level),
                               double(params->precond_dense_levels)};
    // the intermediate tolerance's override is part of what was built
    const char *inner_env = std::getenv("HODBF_CHI_INNER");
    key.push_back(inner_env ? std::atof(inner_env) : -1.0);
    if (params->eps_r && n > 0) key.insert(key.end(), params->eps_r, params->eps_r + 2 * n);
    if (key != g_pp_key) {
      if (!(params->tol_fact > 0 && params->tol_fact < 1)) fail(HODBF_E_ARG, "tol_fact must lie in (0, 1)");
      FwdPlan fp = build_forward_plan(*params);
      fp.ker.tree = &fp.tree;
      auto E = make_host_engine(&fp.tree, 256, programs);
      RbfOpts o;
      o.chi = params->tol_fact;
      // intermediate reconstructions (A22^{-1}, the Schur update, the inner products of
      // the recursion) at 1e-2 chi_fact: their errors are amplified by the inverses
      // the later steps multiply through; HODBF_CHI_INNER overrides
      o.chi_inner = 1e-2 * o.chi;
      if (const char *e = std::getenv("HODBF_CHI_INNER")) o.chi_inner = std::atof(e);
      o.seed = params->seed ^ 0xA5A5A5A5ull;
      const int minl = std::min(params->precond_min_level, fp.tree.depth);
      const int lb = fp.tree.depth - std::min(params->precond_dense_levels, fp.tree.depth);
      if (lb < minl) fail(HODBF_E_ARG, "precond_dense_levels reaches above precond_min_level");
      PrecondBuild pb = invert_hodbf(
          *E, fp.ker, minl, lb, [&](int l) { return forward_offdiag_explicit(fp.tree, fp.bfs, fp.ker, l); }, o);
      g_pp_perm = fp.tree.perm;
      export_precond_build(pb, g_pp_table, g_pp_vals);
      g_pp_stats = {pb.reconstructions, pb.woodbury, pb.stats.sketch_cols, pb.stats.ids,
                    pb.stats.max_rank, pb.stats.applies};
      g_pp_key = key;
    }
    switch (which) {
      case 0:
        pp_export(g_pp_perm.data(), g_pp_perm.size() * 4, buf, bytes);
        break;
      case 3:
        pp_export(g_pp_table.data(), g_pp_table.size() * sizeof(BlockRec), buf, bytes);
        break;
      case 4:
        pp_export(g_pp_vals.data(), g_pp_vals.size() * sizeof(cd), buf, bytes);
        break;
      case 7:
        pp_export(g_pp_stats.data(), g_pp_stats.size() * 8, buf, bytes);
        break;
      default:
        fail(HODBF_E_ARG, "unknown probe selector");
    }
  });
}
