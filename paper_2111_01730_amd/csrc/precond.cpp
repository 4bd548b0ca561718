// Construction of the HOD-BF approximate inverse in the multiplicative form of
// Algorithm 1 (Section III-B):
//     D_tau^{-1} = (I + X_tau) diag(D_tau1^{-1}, D_tau2^{-1}),
//     X_tau = A_tau^{-1} - I,  A_tau = [I, D_tau1^{-1} B_tau1; D_tau2^{-1} B_tau2, I],
// built bottom-up on the device by construct.cpp: leaf inverses dense (host FP64),
// then per level D^{-1} B reconstructed from products with random vectors (line 7) and
// X_tau by the butterfly Sherman-Morrison-Woodbury recursion of Algorithm 2 (line 8).
// The X_tau butterflies (four per node, on the children pairs, L_H - l - 1 levels) are
// packed into one grouped-GEMM program per level.  With precond_dense_levels = d the
// recursion starts from the dense inverses of the level L_H - d nodes' diagonal blocks
// (computed directly, host FP64) instead of the 64-point leaves: the d lowest levels are
// exact, which removes them from the chain of approximate inverses each level's
// reconstruction multiplies through, and their apply is one launch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "construct_dev.h"
#include "pack_sink.h"
#include "precond_host.h"

namespace hodbf {

namespace {

// IEEE binary16 with round to nearest even (inputs are pre-scaled to |v| <= 1).
uint32_t f32_to_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u;
  int32_t e = int32_t((x >> 23) & 0xFF) - 127 + 15;
  uint32_t mant = x & 0x7FFFFFu;
  if (((x >> 23) & 0xFF) == 0xFF) return sign | 0x7C00u | (mant ? 0x200u : 0u);
  if (e >= 31) return sign | 0x7C00u;
  if (e <= 0) {  // subnormal half or zero
    if (e < -10) return sign;
    mant |= 0x800000u;
    const int shift = 14 - e;
    uint32_t h = mant >> shift;
    const uint32_t rem = mant & ((1u << shift) - 1), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (h & 1u))) ++h;
    return sign | h;
  }
  uint32_t h = (uint32_t(e) << 10) | (mant >> 13);
  const uint32_t rem = mant & 0x1FFFu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;  // may carry into the exponent
  return sign | h;
}

uint32_t to_f16_pair(cd v) { return f32_to_f16(float(v.real())) | (f32_to_f16(float(v.imag())) << 16); }

uint32_t to_bf16_pair(cd v) {
  auto cv = [](float f) -> uint32_t {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return u >> 16;  // inf / nan pass through
    u += 0x7FFFu + ((u >> 16) & 1u);                        // round to nearest even
    return u >> 16;
  };
  return cv(float(v.real())) | (cv(float(v.imag())) << 16);
}

}  // namespace

void build_precond(hodbf_op &op, const std::vector<Butterfly> &plan, hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  PrecondData &pd = op.pre;
  const Tree &t = op.tree;
  const int LH = t.depth;
  const auto &p = op.params;
  pd.min_level = std::min(p.precond_min_level, LH);
  const int dl = std::min(p.precond_dense_levels, LH);
  const int lb = LH - dl;
  if (dl > 0 && lb < pd.min_level)
    fail(HODBF_E_ARG, "precond_dense_levels reaches above precond_min_level");
  const bool want32 = (p.precond_prec & HODBF_P_FP32) != 0;
  const bool wantb16 = (p.precond_prec & HODBF_P_BF16) != 0;
  const bool wanth16 = (p.precond_prec & HODBF_P_FP16) != 0;

  // Algorithm 1 on the device; sketch chunks of at most ~2 GiB per multi-vector (complex
  // FP64)
  const int mc = int(std::clamp<int64_t>((int64_t(1) << 31) / (16 * std::max<int64_t>(t.n, 1)), 32, 2048)) & ~31;
  auto E = make_device_engine(&t, st, mc);
  RbfOpts o;
  o.chi = p.tol_fact;
  o.seed = p.seed ^ 0xA5A5A5A5ull;
  // intermediate reconstructions (A22^{-1}, the Schur update, the inner products of
  // the recursion) at 1e-2 chi_fact: their errors are amplified by the inverses
  // the later steps multiply through; HODBF_CHI_INNER overrides
  o.chi_inner = 1e-2 * o.chi;
  if (const char *e = std::getenv("HODBF_CHI_INNER")) o.chi_inner = std::atof(e);
  PrecondBuild pb = invert_hodbf(
      *E, op.ker, pd.min_level, lb,
      [&](int l) { return forward_offdiag_explicit(t, plan, op.ker, l); }, o);
  std::vector<DenseDiag> first = std::move(pb.leaf_inv);
  pb.ops.clear();
  pb.leaf_op.reset();
  E.reset();

  // all factor values, each block divided by its largest component magnitude (the
  // pair's load scale), so that the FP16 copy neither overflows nor underflows
  std::vector<cf> host;
  pd.scales.clear();
  pd.table.clear();
  auto put = [&](const Mat &f, float *scale) -> int64_t {
    const int64_t off = (int64_t(host.size()) + 15) & ~int64_t(15);
    host.resize(size_t(off + int64_t(f.m) * f.n));
    double mx = 0;
    for (const cf &v : f.v)
      mx = std::max({mx, std::abs(double(v.real())), std::abs(double(v.imag()))});
    const float s = mx > 0 ? float(mx) : 1.0f;
    const double inv = 1.0 / double(s);
    for (size_t e = 0; e < f.v.size(); ++e) host[size_t(off) + e] = cf(cd(f.v[e]) * inv);
    *scale = s;
    return off;
  };
  // the first program: dense inverses of the level-lb nodes, each cut into row tiles of
  // at most kTileRows rows that read the node's whole input range
  {
    PackSink pk;
    pk.table = &pd.table;
    for (size_t g = 0; g < first.size(); ++g) {
      const DenseDiag &d = first[g];
      const int m = d.D.m;
      for (const cf &v : d.D.v)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
          fail(HODBF_E_NUMERIC, "non-finite preconditioner factor");
      float scale = 1.0f;
      const int64_t off = put(d.D, &scale);
      pk.table->push_back({0, lb, int64_t(g), 0, 0, 0, 0, 0, m, m, off, m});
      pd.scales.push_back(scale);
      for (int r0 = 0; r0 < m; r0 += kTileRows) {
        Pair pr{};
        pr.f_off = off + r0;
        pr.in_row = d.lo;
        pr.n = m;
        pr.lda = m;
        pr.in_buf = 0;
        pr.scale = scale;
        Seg sg{};
        sg.m = std::min(kTileRows, m - r0);
        sg.p0 = int32_t(pk.pairs.size());
        sg.p1 = sg.p0 + 1;
        sg.map0 = int32_t(pk.rowmap.size());
        sg.map1 = sg.map0 + 1;
        pk.rowmap.push_back({0, d.lo + r0});
        pk.pairs.push_back(pr);
        pk.segs.push_back(sg);
      }
    }
    pk.launches.push_back({0, int64_t(pk.segs.size()), 0, 1});
    upload_program(pd.leaf, pk, st, true, t.n, int64_t(host.size()));
  }
  int maxr = 0;
  pd.levels.clear();
  for (size_t i = 0; i < pb.levels.size(); ++i) {
    const int l = lb - 1 - int(i);
    std::vector<const Butterfly *> ptrs;
    for (const Butterfly &bf : pb.levels[i]) {
      ptrs.push_back(&bf);
      for (auto &v : bf.V0) maxr = std::max(maxr, v.m);
      for (int lv = 1; lv <= bf.L; ++lv)
        for (auto &w : bf.W[size_t(lv)]) maxr = std::max(maxr, w.m);
    }
    PackSink pk;
    pk.table = &pd.table;
    pk.scales = &pd.scales;
    pk.put_host = put;
    pack_group(pk, t, ptrs, false, 1, [](const Butterfly &bf, int64_t *md) {
      md[0] = bf.hod_level - 1;
      md[1] = bf.tau;
      md[2] = bf.ca;
      md[3] = bf.cb;
    });
    PrecondLevel lv;
    lv.level = l;
    upload_program(lv.prog, pk, st, true, t.n, int64_t(host.size()));
    pd.levels.push_back(std::move(lv));
  }
  for (const cf &v : host)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
      fail(HODBF_E_NUMERIC, "non-finite preconditioner factor");
  // arenas
  const size_t count = host.size();
  if (want32) {
    static_assert(sizeof(cf) == sizeof(float2), "complex<float> is two floats");
    pd.F32.upload(host.data(), count * sizeof(float2), st);
  }
  if (wantb16) {
    std::vector<uint32_t> f(count);
    for (size_t i = 0; i < count; ++i) f[i] = to_bf16_pair(cd(host[i]));
    pd.BF16.upload(f.data(), count * sizeof(uint32_t), st);
  }
  if (wanth16) {
    std::vector<uint32_t> f(count);
    for (size_t i = 0; i < count; ++i) f[i] = to_f16_pair(cd(host[i]));
    pd.F16.upload(f.data(), count * sizeof(uint32_t), st);
  }
  const size_t total = op.fwdF.bytes + pd.F32.bytes + pd.BF16.bytes + pd.F16.bytes;
  if (p.hbm_budget && total > p.hbm_budget) fail(HODBF_E_NOMEM, "operator exceeds hbm_budget");
  int64_t ent = 0;
  for (auto &r : pd.table) ent += r.m * r.n;
  pd.entries = ent;
  pd.max_rank = maxr;
  // default arithmetic: the FP32 copy on split-BF16 MFMA when it is stored (it
  // preconditions like FP32 arithmetic at a lower cost), else FP16, else BF16
  pd.default_ft = want32 ? FT_C64_S3 : (wanth16 ? FT_F16 : FT_BF16);
  pd.present = true;
  pd.reconstructions = pb.reconstructions;
  pd.sketch_cols = pb.stats.sketch_cols;
  op.id_count += pb.stats.ids;
  pd.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  logf("preconditioner: %lld entries, largest rank %d, %lld reconstructions, %lld sketch columns, "
       "%.2f s", (long long)ent, maxr, (long long)pb.reconstructions, (long long)pb.stats.sketch_cols,
       pd.seconds);
}

}  // namespace hodbf
