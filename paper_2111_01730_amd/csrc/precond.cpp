// Construction of the HOD-BF approximate inverse in the multiplicative form of
// Algorithm 1 (Section III-B):
//     D_tau^{-1} = (I + X_tau) diag(D_tau1^{-1}, D_tau2^{-1}),
//     X_tau = A_tau^{-1} - I = D_tau^{-1} diag(D_tau1, D_tau2) - I.
// The paper reaches X_tau through randomized butterfly reconstruction and the
// butterfly Sherman-Morrison-Woodbury recursion.  Here each X_tau is formed from its
// definition on the GPU (dense LU of D_tau = Z(tau, tau) with rocSOLVER, solved
// against diag(D_tau1, D_tau2)), then its four child blocks X_tau(tau_i, tau_j) are
// compressed into butterflies with L_H - l - 1 levels by the same sampled-row nested
// ID used for Z, at tolerance chi_fact.  Leaf inverses are dense.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "pack_sink.h"

namespace hodbf {

void build_butterflies(const EntrySource &src, const Tree &t, std::vector<Butterfly> &bfs,
                       double chi, uint64_t seed, int64_t *id_count);

namespace {

void rb_check(rocblas_status s, const char *what) {
  if (s != rocblas_status_success)
    fail(HODBF_E_HIP, std::string(what) + " failed with rocblas status " + std::to_string(int(s)));
}

// Dense in-place inverse of a small complex matrix (column-major) by Gauss-Jordan
// elimination with partial pivoting.
void small_inverse(std::vector<cd> &A, int n) {
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) piv[i] = i;
  std::vector<cd> I(size_t(n) * n, cd(0, 0));
  for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[size_t(c) * n + r]) > std::abs(A[size_t(c) * n + p])) p = r;
    if (!(std::abs(A[size_t(c) * n + p]) > 0)) fail(HODBF_E_NUMERIC, "singular leaf block");
    if (p != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[size_t(k) * n + p], A[size_t(k) * n + c]);
        std::swap(I[size_t(k) * n + p], I[size_t(k) * n + c]);
      }
    const cd inv = 1.0 / A[size_t(c) * n + c];
    for (int k = 0; k < n; ++k) {
      A[size_t(k) * n + c] *= inv;
      I[size_t(k) * n + c] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cd f = A[size_t(c) * n + r];
      if (f == cd(0, 0)) continue;
      for (int k = 0; k < n; ++k) {
        A[size_t(k) * n + r] -= f * A[size_t(k) * n + c];
        I[size_t(k) * n + r] -= f * I[size_t(k) * n + c];
      }
    }
  }
  A.swap(I);
}

// Entries of a dense host block X (column-major, rows/cols offset by lo).
struct DenseSource final : EntrySource {
  const cd *X = nullptr;
  int64_t n = 0, lo = 0;
  void fill(const int32_t *rows, int nr, const int32_t *cols, int nc, cd *out) const override {
    for (int c = 0; c < nc; ++c) {
      const cd *col = X + size_t(cols[c] - lo) * size_t(n);
      for (int r = 0; r < nr; ++r) out[size_t(c) * nr + r] = col[rows[r] - lo];
    }
  }
};

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

// X + I = Z(tau,tau)^{-1} diag(Z(tau1,tau1), Z(tau2,tau2)) on the device; returns X on the host.
static void dense_x(hodbf_op &op, rocblas_handle rh, int l, int64_t tau, std::vector<cd> &Xh,
                    hipStream_t st) {
  const Tree &t = op.tree;
  const int32_t lo = t.node_lo(l, tau), hi = t.node_hi(l, tau);
  const int64_t n = hi - lo;
  const int32_t mid = t.node_lo(l + 1, 2 * tau + 1);
  // column jobs for K1 (FP64): the whole tau x tau block, column chunks of 64
  std::vector<EntryJob> jobs;
  std::vector<int32_t> cols(static_cast<size_t>(n));
  for (int64_t k = 0; k < n; ++k) cols[size_t(k)] = int32_t(lo + k);
  for (int64_t c0 = 0; c0 < n; c0 += 64) {
    const int64_t nc = std::min<int64_t>(64, n - c0);
    jobs.push_back({c0 * n, lo, int32_t(n), int32_t(c0), int32_t(nc)});
  }
  DevBuf dj, dc, A, B, piv, info;
  dj.upload(jobs.data(), jobs.size() * sizeof(EntryJob), st);
  dc.upload(cols.data(), cols.size() * sizeof(int32_t), st);
  A.alloc(size_t(n) * n * sizeof(double2));
  B.alloc(size_t(n) * n * sizeof(double2));
  piv.alloc(size_t(n) * sizeof(int64_t));
  info.alloc(sizeof(int64_t));
  const double2 k2S = make_double2(op.ker.k2S.real(), op.ker.k2S.imag());
  launch_entries(dj.as<EntryJob>(), int64_t(jobs.size()), dc.as<int32_t>(), op.dev.xyz.as<short4>(),
                 op.dev.inv_eps.as<double2>(), op.dev.kappa.as<double2>(), op.ker.kh, k2S, nullptr,
                 A.as<double2>(), st);
  HIPCHK(hipGetLastError());
  // B = diag(Z(tau1, tau1), Z(tau2, tau2)): copy the two diagonal blocks of A
  HIPCHK(hipMemsetAsync(B.p, 0, B.bytes, st));
  const int64_t n1 = mid - lo, n2 = hi - mid;
  HIPCHK(hipMemcpy2DAsync(B.p, size_t(n) * 16, A.p, size_t(n) * 16, size_t(n1) * 16, size_t(n1),
                          hipMemcpyDeviceToDevice, st));
  const size_t off2 = (size_t(n1) * n + n1) * 16;
  HIPCHK(hipMemcpy2DAsync(B.as<char>() + off2, size_t(n) * 16, A.as<char>() + off2,
                          size_t(n) * 16, size_t(n2) * 16, size_t(n2), hipMemcpyDeviceToDevice, st));
  rb_check(rocblas_set_stream(rh, st), "rocblas_set_stream");
  rb_check(rocsolver_zgetrf_64(rh, n, n, A.as<rocblas_double_complex>(), n, piv.as<int64_t>(),
                               info.as<int64_t>()),
           "rocsolver_zgetrf_64");
  int64_t hinfo = 0;
  HIPCHK(hipMemcpyAsync(&hinfo, info.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hinfo != 0) fail(HODBF_E_NUMERIC, "singular diagonal block in the preconditioner");
  rb_check(rocsolver_zgetrs_64(rh, rocblas_operation_none, n, n, A.as<rocblas_double_complex>(), n,
                               piv.as<int64_t>(), B.as<rocblas_double_complex>(), n),
           "rocsolver_zgetrs_64");
  Xh.resize(size_t(n) * n);
  HIPCHK(hipMemcpyAsync(Xh.data(), B.p, B.bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) Xh[size_t(i) * n + i] -= 1.0;
  for (auto &v : Xh)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
      fail(HODBF_E_NUMERIC, "non-finite preconditioner factor");
}

// Z(tau, tau)^{-1} of a level-l node on the device (complex FP64 LU); returned column-major
// on the host.
static void dense_inverse(hodbf_op &op, rocblas_handle rh, int l, int64_t tau,
                          std::vector<cd> &Xh, hipStream_t st) {
  const Tree &t = op.tree;
  const int32_t lo = t.node_lo(l, tau), hi = t.node_hi(l, tau);
  const int64_t n = hi - lo;
  std::vector<EntryJob> jobs;
  std::vector<int32_t> cols(static_cast<size_t>(n));
  for (int64_t k = 0; k < n; ++k) cols[size_t(k)] = int32_t(lo + k);
  for (int64_t c0 = 0; c0 < n; c0 += 64) {
    const int64_t nc = std::min<int64_t>(64, n - c0);
    jobs.push_back({c0 * n, lo, int32_t(n), int32_t(c0), int32_t(nc)});
  }
  std::vector<cd> eye(size_t(n) * n, cd(0.0, 0.0));
  for (int64_t i = 0; i < n; ++i) eye[size_t(i) * n + i] = 1.0;
  DevBuf dj, dc, A, B, piv, info;
  dj.upload(jobs.data(), jobs.size() * sizeof(EntryJob), st);
  dc.upload(cols.data(), cols.size() * sizeof(int32_t), st);
  B.upload(eye.data(), eye.size() * sizeof(cd), st);
  A.alloc(size_t(n) * n * sizeof(double2));
  piv.alloc(size_t(n) * sizeof(int64_t));
  info.alloc(sizeof(int64_t));
  const double2 k2S = make_double2(op.ker.k2S.real(), op.ker.k2S.imag());
  launch_entries(dj.as<EntryJob>(), int64_t(jobs.size()), dc.as<int32_t>(), op.dev.xyz.as<short4>(),
                 op.dev.inv_eps.as<double2>(), op.dev.kappa.as<double2>(), op.ker.kh, k2S, nullptr,
                 A.as<double2>(), st);
  HIPCHK(hipGetLastError());
  rb_check(rocblas_set_stream(rh, st), "rocblas_set_stream");
  rb_check(rocsolver_zgetrf_64(rh, n, n, A.as<rocblas_double_complex>(), n, piv.as<int64_t>(),
                               info.as<int64_t>()),
           "rocsolver_zgetrf_64");
  int64_t hinfo = 0;
  HIPCHK(hipMemcpyAsync(&hinfo, info.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hinfo != 0) fail(HODBF_E_NUMERIC, "singular diagonal block in the preconditioner");
  rb_check(rocsolver_zgetrs_64(rh, rocblas_operation_none, n, n, A.as<rocblas_double_complex>(), n,
                               piv.as<int64_t>(), B.as<rocblas_double_complex>(), n),
           "rocsolver_zgetrs_64");
  Xh.resize(size_t(n) * n);
  HIPCHK(hipMemcpyAsync(Xh.data(), B.p, B.bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (auto &v : Xh)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
      fail(HODBF_E_NUMERIC, "non-finite preconditioner factor");
}

void build_precond(hodbf_op &op, hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  PrecondData &pd = op.pre;
  const Tree &t = op.tree;
  const int LH = t.depth;
  const auto &p = op.params;
  pd.min_level = std::min(p.precond_min_level, LH);
  // level of the dense diagonal inverses that start the product: the leaves, or, with
  // precond_dense_levels = d, the level L_H - d nodes (their exact inverses are what the
  // leaf inverses and the d lowest levels of X_tau compose to)
  const int dl = std::min(p.precond_dense_levels, LH);
  const int lb = LH - dl;
  if (dl > 0 && lb < pd.min_level)
    fail(HODBF_E_ARG, "precond_dense_levels reaches above precond_min_level");
  const bool want32 = (p.precond_prec & HODBF_P_FP32) != 0;
  const bool wantb16 = (p.precond_prec & HODBF_P_BF16) != 0;
  const bool wanth16 = (p.precond_prec & HODBF_P_FP16) != 0;
  // all factor values, each block divided by its largest component magnitude (the
  // pair's load scale), so that the FP16 copy neither overflows nor underflows
  std::vector<cf> host;
  pd.scales.clear();
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
  rocblas_handle rh = nullptr;
  rb_check(rocblas_create_handle(&rh), "rocblas_create_handle");
  struct HandleGuard {
    rocblas_handle h;
    ~HandleGuard() { rocblas_destroy_handle(h); }
  } guard{rh};
  // the first program: dense inverses of the diagonal blocks of the level-lb nodes (the
  // leaves: FP64 on the host; larger nodes: FP64 LU on the device), each cut into row
  // tiles of at most kTileRows rows that read the node's whole input range
  {
    PackSink pk;
    pk.table = &pd.table;
    const int64_t nnode = int64_t(1) << lb;
    for (int64_t g = 0; g < nnode; ++g) {
      const int32_t lo = t.node_lo(lb, g), hi = t.node_hi(lb, g);
      const int m = hi - lo;
      std::vector<cd> Dv;
      if (lb == LH) {
        Dv.resize(size_t(m) * m);
        for (int c = 0; c < m; ++c)
          for (int r = 0; r < m; ++r) Dv[size_t(c) * m + r] = op.ker.entry(lo + r, lo + c);
        small_inverse(Dv, m);
      } else {
        dense_inverse(op, rh, lb, g, Dv, st);
      }
      Mat D;
      D.m = D.n = m;
      D.v.assign(Dv.begin(), Dv.end());
      float scale = 1.0f;
      const int64_t off = put(D, &scale);
      pk.table->push_back({0, lb, g, 0, 0, 0, 0, 0, m, m, off, m});
      pd.scales.push_back(scale);
      for (int r0 = 0; r0 < m; r0 += kTileRows) {
        Pair pr{};
        pr.f_off = off + r0;
        pr.in_row = lo;
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
        pk.rowmap.push_back({0, lo + r0});
        pk.pairs.push_back(pr);
        pk.segs.push_back(sg);
      }
    }
    pk.launches.push_back({0, int64_t(pk.segs.size()), 0, 1});
    upload_program(pd.leaf, pk, st);
  }
  int maxr = 0;
  int64_t ids = 0;
  for (int l = lb - 1; l >= pd.min_level; --l) {
    std::vector<Butterfly> bfs;
    for (int64_t tau = 0; tau < (int64_t(1) << l); ++tau) {
      std::vector<cd> Xh;
      dense_x(op, rh, l, tau, Xh, st);
      if (t.node_hi(l, tau) - t.node_lo(l, tau) >= 4096)
        logf("  dense X for level %d node %lld ready, %.2f s", l, (long long)tau,
             std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      DenseSource src;
      src.tree = &t;
      src.X = Xh.data();
      src.n = t.node_hi(l, tau) - t.node_lo(l, tau);
      src.lo = t.node_lo(l, tau);
      std::vector<Butterfly> four;
      for (int ca = 0; ca < 2; ++ca)
        for (int cb = 0; cb < 2; ++cb) {
          Butterfly bf;
          bf.hod_level = l + 1;
          bf.oi = 2 * tau + ca;
          bf.si = 2 * tau + cb;
          bf.ca = ca;
          bf.cb = cb;
          bf.tau = tau;
          bf.L = LH - l - 1;
          four.push_back(std::move(bf));
        }
      build_butterflies(src, t, four, p.tol_fact, p.seed ^ (uint64_t(l) << 40) ^ uint64_t(tau),
                        &ids);
      for (auto &bf : four) {
        const int64_t na = int64_t(1) << bf.L;
        bf.B.resize(size_t(na));
        for (int64_t a = 0; a < na; ++a) {
          const int32_t r0 = t.node_lo(LH, (bf.oi << bf.L) + a), r1 = t.node_hi(LH, (bf.oi << bf.L) + a);
          const auto &sk = bf.bskel[size_t(a)];
          Mat &B = bf.B[size_t(a)];
          B.m = r1 - r0;
          B.n = int(sk.size());
          std::vector<cd> Bv(size_t(B.m) * B.n);
          std::vector<int32_t> rows(static_cast<size_t>(B.m));
          for (int i = 0; i < B.m; ++i) rows[size_t(i)] = r0 + i;
          if (B.n) src.fill(rows.data(), B.m, sk.data(), B.n, Bv.data());
          B.v.assign(Bv.begin(), Bv.end());
        }
        for (auto &v : bf.V0) maxr = std::max(maxr, v.m);
        for (int lv = 1; lv <= bf.L; ++lv)
          for (auto &w : bf.W[size_t(lv)]) maxr = std::max(maxr, w.m);
        bf.bskel.clear();
        bfs.push_back(std::move(bf));
      }
    }
    PackSink pk;
    pk.table = &pd.table;
    pk.scales = &pd.scales;
    pk.put_host = put;
    std::vector<const Butterfly *> ptrs;
    for (auto &bf : bfs) ptrs.push_back(&bf);
    pack_group(pk, t, ptrs, false, 1, [](const Butterfly &bf, int64_t *md) {
      md[0] = bf.hod_level - 1;
      md[1] = bf.tau;
      md[2] = bf.ca;
      md[3] = bf.cb;
    });
    logf("preconditioner level %d: %lld nodes, %.2f s so far", l, (long long)(int64_t(1) << l),
         std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    PrecondLevel lv;
    lv.level = l;
    upload_program(lv.prog, pk, st);
    pd.levels.push_back(std::move(lv));
  }
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
  op.id_count += ids;
  pd.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace hodbf
