// C ABI of the hodbf library: construction, applies, export and error handling.
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>

#include "pack_sink.h"
#include "precond_host.h"

namespace hodbf {

// ---------------------------------------------------------------------------
// errors
static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

[[noreturn]] void fail(hodbf_status code, const std::string &msg) { throw Error{code, msg}; }

void logf(const char *fmt, ...) {
  // read at every message (cheap next to what is logged) so a caller can switch it on
  // for one long call
  const char *e = std::getenv("HODBF_LOG");
  if (!(e && *e && std::strcmp(e, "0") != 0)) return;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "[hodbf] ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  std::fflush(stderr);
  va_end(ap);
}

void hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  const hodbf_status code = (e == hipErrorOutOfMemory) ? HODBF_E_NOMEM : HODBF_E_HIP;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
static hodbf_status guarded(F &&f) {
  return hodbf_guarded(std::forward<F>(f));
}

// ---------------------------------------------------------------------------
// device memory: the caller's allocator hook when one is installed, else the HIP runtime
namespace {
struct AllocHook {
  hodbf_alloc_fn alloc = nullptr;
  hodbf_free_fn release = nullptr;
  void *ctx = nullptr;
};
std::mutex g_hook_mu;
AllocHook g_hook;
AllocHook current_hook() {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  return g_hook;
}
}  // namespace

void DevBuf::reset() {
  if (p) {
    if (release) release(p, ctx);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
  release = nullptr;
  ctx = nullptr;
}
void DevBuf::alloc(size_t nbytes) {
  reset();
  if (nbytes == 0) return;
  const AllocHook h = current_hook();
  if (h.alloc) {
    p = h.alloc(nbytes, nullptr, h.ctx);
    if (!p) fail(HODBF_E_NOMEM, "allocator hook returned NULL");
    release = h.release;
    ctx = h.ctx;
  } else {
    HIPCHK(hipMalloc(&p, nbytes));
  }
  bytes = nbytes;
}
void DevBuf::upload(const void *src, size_t nbytes, hipStream_t st) {
  alloc(nbytes);
  if (nbytes) {
    HIPCHK(hipMemcpyAsync(p, src, nbytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
}

Scratch::Scratch(size_t bytes, hipStream_t st) : st_(st) {
  if (bytes == 0) bytes = 256;
  const AllocHook h = current_hook();
  if (h.alloc) {
    p_ = h.alloc(bytes, st, h.ctx);
    if (!p_) fail(HODBF_E_NOMEM, "allocator hook returned NULL");
    release_ = h.release;
    ctx_ = h.ctx;
  } else {
    HIPCHK(hipMallocAsync(&p_, bytes, st));
  }
}
Scratch::~Scratch() {
  if (!p_) return;
  if (release_) release_(p_, ctx_);
  else (void)hipFreeAsync(p_, st_);
}


// ---------------------------------------------------------------------------
// programs
void run_program(const Program &prog, const void *F, int ftype, const float2 *X, float2 *T,
                 float2 *OUT, int R, hipStream_t st) {
  for (const Launch &ln : prog.launches) {
    launch_grouped(prog.segs.as<Seg>(), prog.pairs.as<Pair>(), prog.rowmap.as<RowMap>(), ln.s0,
                   ln.ns, ln.cls, F, ftype, X, T, ln.out ? OUT : T, R, ln.beta, st);
  }
}

int64_t forward_work_rows(const hodbf_op &op) { return op.fwd.t_rows; }

void apply_forward_tree(const hodbf_op &op, const float2 *x, float2 *y, float2 *work, int R,
                        hipStream_t st, int ftype) {
  run_program(op.fwd, op.fwdF.p, ftype, x, work, y, R, st);
}

int64_t precond_work_rows(const hodbf_op &op) {
  int64_t r = 0;
  for (auto &lv : op.pre.levels) r = std::max(r, lv.prog.t_rows);
  return r;
}

void apply_precond_tree(const hodbf_op &op, int ftype, const float2 *x, float2 *z, float2 *work,
                        int R, hipStream_t st) {
  const void *F = ftype == FT_BF16 ? op.pre.BF16.p : (ftype == FT_F16 ? op.pre.F16.p : op.pre.F32.p);
  // z = blockdiag(D_leaf^{-1}) x, then z(tau) += X_tau z(tau) level by level to the root
  run_program(op.pre.leaf, F, ftype, x, work, z, R, st);
  for (const PrecondLevel &lv : op.pre.levels) run_program(lv.prog, F, ftype, z, work, z, R, st);
}

// ---------------------------------------------------------------------------
static void upload_geometry(hodbf_op &op, hipStream_t st) {
  const Tree &t = op.tree;
  op.dev.perm.upload(t.perm.data(), t.perm.size() * sizeof(int32_t), st);
  std::vector<int32_t> tpos(t.perm.size());
  for (size_t i = 0; i < t.perm.size(); ++i) tpos[size_t(t.perm[i])] = int32_t(i);
  op.dev.tpos.upload(tpos.data(), tpos.size() * sizeof(int32_t), st);
  std::vector<short4> xyz(static_cast<size_t>(t.n));
  for (int64_t i = 0; i < t.n; ++i) xyz[size_t(i)] = make_short4(t.cx[size_t(i)], t.cy[size_t(i)], t.cz[size_t(i)], 0);
  op.dev.xyz.upload(xyz.data(), xyz.size() * sizeof(short4), st);
  std::vector<double2> ie(static_cast<size_t>(t.n)), ka(static_cast<size_t>(t.n));
  for (int64_t i = 0; i < t.n; ++i) {
    ie[size_t(i)] = make_double2(op.ker.inv_eps[size_t(i)].real(), op.ker.inv_eps[size_t(i)].imag());
    ka[size_t(i)] = make_double2(op.ker.kappa[size_t(i)].real(), op.ker.kappa[size_t(i)].imag());
  }
  op.dev.inv_eps.upload(ie.data(), ie.size() * sizeof(double2), st);
  op.dev.kappa.upload(ka.data(), ka.size() * sizeof(double2), st);
}

static int64_t align16(int64_t x) { return (x + 15) & ~int64_t(15); }

static void pack_forward(hodbf_op &op, FwdPlan &fp, hipStream_t st) {
  std::vector<float2> host;  // V0 / W values (region 1)
  std::vector<std::pair<int64_t, int64_t>> dev_blocks;
  int64_t dev_size = 0;
  std::vector<EntryJob> jobs;
  std::vector<int32_t> jobcols;
  PackSink pk;
  pk.table = &op.fwd_table;
  pk.put_host = [&](const Mat &f, float *scale) -> int64_t {
    *scale = 1.0f;
    const int64_t off = align16(int64_t(host.size()));
    host.resize(size_t(off + int64_t(f.m) * f.n), make_float2(0.f, 0.f));
    for (size_t e = 0; e < f.v.size(); ++e)
      host[size_t(off) + e] = make_float2(float(f.v[e].real()), float(f.v[e].imag()));
    return off;
  };
  // device-generated blocks get provisional offsets kDevRegion + off in region 2, rebased
  // below (a positive bias, so row offsets added while packing carry over)
  constexpr int64_t kDevRegion = int64_t(1) << 60;
  pk.reserve_dev = [&](int64_t m, int64_t n) -> int64_t {
    const int64_t off = align16(dev_size);
    dev_size = off + m * n;
    return kDevRegion + off;
  };
  pk.jobs = &jobs;
  pk.jobcols = &jobcols;
  std::vector<const Butterfly *> bfs;
  for (auto &bf : fp.bfs) bfs.push_back(&bf);
  pack_group(pk, op.tree, bfs, true, 0, [](const Butterfly &bf, int64_t *md) {
    md[0] = bf.hod_level;
    md[1] = bf.oi;
    md[2] = 0;
    md[3] = 0;
  });
  const int64_t base2 = align16(int64_t(host.size()));
  auto rebase = [&](int64_t off) { return off >= kDevRegion ? base2 + (off - kDevRegion) : off; };
  for (auto &p : pk.pairs) p.f_off = rebase(p.f_off);
  for (auto &j : jobs) j.f_off = rebase(j.f_off);
  for (auto &r : op.fwd_table) r.off = rebase(r.off);
  const int64_t total = base2 + dev_size;
  const size_t bytes = size_t(total) * sizeof(float2);
  if (op.params.hbm_budget && bytes > op.params.hbm_budget)
    fail(HODBF_E_NOMEM, "forward operator exceeds hbm_budget");
  op.fwdF.alloc(bytes);
  if (!host.empty())
    HIPCHK(hipMemcpyAsync(op.fwdF.p, host.data(), host.size() * sizeof(float2),
                          hipMemcpyHostToDevice, st));
  DevBuf djobs, dcols;
  djobs.upload(jobs.data(), jobs.size() * sizeof(EntryJob), st);
  dcols.upload(jobcols.data(), std::max<size_t>(1, jobcols.size()) * sizeof(int32_t), st);
  const double2 k2S = make_double2(op.ker.k2S.real(), op.ker.k2S.imag());
  launch_entries(djobs.as<EntryJob>(), int64_t(jobs.size()), dcols.as<int32_t>(),
                 op.dev.xyz.as<short4>(), op.dev.inv_eps.as<double2>(), op.dev.kappa.as<double2>(),
                 op.ker.kh, k2S, op.fwdF.as<float2>(), nullptr, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  upload_program(op.fwd, pk, st, true, op.n, total);
  int64_t ent = 0;
  for (auto &r : op.fwd_table) ent += r.m * r.n;
  op.fwd_entries = ent;
}

}  // namespace hodbf

using namespace hodbf;

extern "C" {

hodbf_status hodbf_build(const hodbf_build_params *params, hodbf_op **out) {
  return guarded([&] {
    if (!params || !out) fail(HODBF_E_ARG, "NULL argument");
    *out = nullptr;
    hipStream_t st = static_cast<hipStream_t>(params->stream);
    auto t0 = std::chrono::steady_clock::now();
    FwdPlan fp = build_forward_plan(*params);
    logf("forward plan: N=%lld, L_H=%d, %lld IDs, max rank %d, %.2f s", (long long)fp.tree.n,
         fp.tree.depth, (long long)fp.id_count, fp.max_rank,
         std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    std::unique_ptr<hodbf_op> op(new hodbf_op());
    op->params = *params;
    op->params.eps_r = nullptr;
    op->n = fp.tree.n;
    op->tree = std::move(fp.tree);
    op->ker = fp.ker;
    op->ker.tree = &op->tree;
    op->max_rank = fp.max_rank;
    op->id_count = fp.id_count;
    upload_geometry(*op, st);
    pack_forward(*op, fp, st);
    op->build_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (params->precond_prec != HODBF_P_NONE) build_precond(*op, fp.bfs, st);
    fp.bfs.clear();
    *out = op.release();
  });
}

void hodbf_free(hodbf_op *op) { delete op; }

hodbf_status hodbf_set_allocator(hodbf_alloc_fn alloc, hodbf_free_fn release, void *ctx) {
  return guarded([&] {
    if (alloc && !release) fail(HODBF_E_ARG, "allocator hook without a release function");
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_hook.alloc = alloc;
    g_hook.release = alloc ? release : nullptr;
    g_hook.ctx = alloc ? ctx : nullptr;
  });
}

const char *hodbf_last_error(void) { return g_last_error.c_str(); }

static void check_vec_args(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype, const void *x,
                           int64_t ldx, const void *y, int64_t ldy) {
  if (!op) fail(HODBF_E_ARG, "NULL operator");
  if (nrhs < 0) fail(HODBF_E_ARG, "nrhs < 0");
  if (dtype != HODBF_C64 && dtype != HODBF_C128) fail(HODBF_E_ARG, "unknown dtype");
  if (nrhs == 0) return;
  if (!x || !y) fail(HODBF_E_ARG, "NULL vector");
  if (ldx < op->n || ldy < op->n) fail(HODBF_E_ARG, "leading dimension < N");
  const size_t es = dtype == HODBF_C128 ? 16 : 8;
  const char *xb = static_cast<const char *>(x), *yb = static_cast<const char *>(y);
  const char *xe = xb + es * size_t(ldx * (nrhs - 1) + op->n);
  const char *ye = yb + es * size_t(ldy * (nrhs - 1) + op->n);
  if (xb < ye && yb < xe) fail(HODBF_E_ARG, "x and y overlap");
}

hodbf_status hodbf_apply(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype, const void *x,
                         int64_t ldx, void *y, int64_t ldy, void *stream) {
  return guarded([&] {
    check_vec_args(op, nrhs, dtype, x, ldx, y, ldy);
    if (nrhs == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = op->n;
    const size_t vbytes = size_t(n) * nrhs * sizeof(float2);
    const size_t wbytes = size_t(forward_work_rows(*op)) * nrhs * sizeof(float2);
    const Scratch scr(2 * vbytes + wbytes, st);
    char *buf = scr.as<char>();
    float2 *xt = reinterpret_cast<float2 *>(buf);
    float2 *yt = reinterpret_cast<float2 *>(buf + vbytes);
    float2 *wk = reinterpret_cast<float2 *>(buf + 2 * vbytes);
    const bool c128 = dtype == HODBF_C128;
    launch_gather(x, c128, ldx, xt, false, op->dev.tpos.as<int32_t>(), n, nrhs, st);
    apply_forward_tree(*op, xt, yt, wk, nrhs, st);
    launch_scatter(yt, false, y, c128, ldy, op->dev.perm.as<int32_t>(), n, nrhs, st);
    HIPCHK(hipGetLastError());
  });
}

hodbf_status hodbf_precond_apply(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype,
                                 const void *x, int64_t ldx, void *y, int64_t ldy,
                                 void *stream) {
  return guarded([&] {
    check_vec_args(op, nrhs, dtype, x, ldx, y, ldy);
    if (!op->pre.present) fail(HODBF_E_STATE, "operator was built without a preconditioner");
    if (nrhs == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = op->n;
    const size_t vbytes = size_t(n) * nrhs * sizeof(float2);
    const size_t wbytes = size_t(precond_work_rows(*op)) * nrhs * sizeof(float2);
    const Scratch scr(2 * vbytes + wbytes, st);
    char *buf = scr.as<char>();
    float2 *xt = reinterpret_cast<float2 *>(buf);
    float2 *zt = reinterpret_cast<float2 *>(buf + vbytes);
    float2 *wk = reinterpret_cast<float2 *>(buf + 2 * vbytes);
    const bool c128 = dtype == HODBF_C128;
    launch_gather(x, c128, ldx, xt, false, op->dev.tpos.as<int32_t>(), n, nrhs, st);
    apply_precond_tree(*op, op->pre.default_ft, xt, zt, wk, nrhs, st);
    launch_scatter(zt, false, y, c128, ldy, op->dev.perm.as<int32_t>(), n, nrhs, st);
    HIPCHK(hipGetLastError());
  });
}

hodbf_status hodbf_apply_tree(const hodbf_op *op, int32_t which, int32_t nrhs, const void *x,
                              void *y, void *stream) {
  return guarded([&] {
    if (!op || nrhs < 0 || which < 0 || which > 6) fail(HODBF_E_ARG, "bad operator, nrhs or which");
    if (nrhs == 0) return;
    if (!x || !y) fail(HODBF_E_ARG, "NULL vector");
    const size_t vb = size_t(op->n) * nrhs * sizeof(float2);
    const char *xb = static_cast<const char *>(x), *yb = static_cast<const char *>(y);
    if (xb < yb + vb && yb < xb + vb) fail(HODBF_E_ARG, "x and y overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool fwd = which == 0 || which == 5;
    int ft = which == 5 ? FT_C64_S3 : FT_C64;
    if (!fwd) {
      if (!op->pre.present) fail(HODBF_E_STATE, "operator was built without a preconditioner");
      ft = which == 1 ? op->pre.default_ft
                      : (which == 2 ? FT_C64 : (which == 3 ? FT_BF16 : (which == 4 ? FT_F16 : FT_C64_S3)));
      if ((ft == FT_C64 || ft == FT_C64_S3) && !op->pre.F32.p)
        fail(HODBF_E_STATE, "no FP32 preconditioner copy");
      if (ft == FT_BF16 && !op->pre.BF16.p) fail(HODBF_E_STATE, "no BF16 preconditioner copy");
      if (ft == FT_F16 && !op->pre.F16.p) fail(HODBF_E_STATE, "no FP16 preconditioner copy");
    }
    const int64_t rows = fwd ? forward_work_rows(*op) : precond_work_rows(*op);
    const Scratch scr(size_t(std::max<int64_t>(rows, 1)) * nrhs * 8, st);
    float2 *wk = scr.as<float2>();
    if (fwd)
      apply_forward_tree(*op, static_cast<const float2 *>(x), static_cast<float2 *>(y), wk, nrhs, st,
                         ft);
    else
      apply_precond_tree(*op, ft, static_cast<const float2 *>(x), static_cast<float2 *>(y), wk, nrhs, st);
    HIPCHK(hipGetLastError());
  });
}

hodbf_status hodbf_plane_wave(const hodbf_op *op, int32_t nrhs, const double *dirs, void *b,
                              int64_t ldb, void *stream) {
  return guarded([&] {
    if (!op || nrhs < 0) fail(HODBF_E_ARG, "bad operator or nrhs");
    if (nrhs == 0) return;
    if (!dirs || !b || ldb < op->n) fail(HODBF_E_ARG, "bad dirs / b / ldb");
    for (int i = 0; i < 3 * nrhs; ++i)
      if (!std::isfinite(dirs[i])) fail(HODBF_E_ARG, "non-finite direction");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Scratch scr(sizeof(double) * 3 * nrhs, st);
    double *dd = scr.as<double>();
    HIPCHK(hipMemcpyAsync(dd, dirs, sizeof(double) * 3 * nrhs, hipMemcpyHostToDevice, st));
    const auto &p = op->params;
    launch_plane_wave(dd, nrhs, p.nx, p.ny, p.nz, p.h, p.k0, static_cast<double2 *>(b), ldb, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
  });
}

hodbf_status hodbf_stats(const hodbf_op *op, hodbf_stats_t *s) {
  return guarded([&] {
    if (!op || !s) fail(HODBF_E_ARG, "NULL argument");
    std::memset(s, 0, sizeof(*s));
    s->n = op->n;
    s->levels = op->tree.depth;
    s->leaves = 1 << op->tree.depth;
    s->max_rank = op->max_rank;
    s->precond_max_rank = op->pre.max_rank;
    s->entries_fwd = op->fwd_entries;
    s->entries_pre = op->pre.entries;
    s->bytes_fwd = int64_t(op->fwdF.bytes);
    s->bytes_pre = int64_t(op->pre.F32.bytes + op->pre.BF16.bytes + op->pre.F16.bytes);
    s->bytes_total = s->bytes_fwd + s->bytes_pre + int64_t(op->fwd.segs.bytes + op->fwd.pairs.bytes) +
                     int64_t(op->dev.perm.bytes + op->dev.tpos.bytes + op->dev.xyz.bytes + op->dev.inv_eps.bytes +
                             op->dev.kappa.bytes);
    s->fwd_stages = int32_t(op->fwd.launches.size());
    int ps = int(op->pre.leaf.launches.size());
    for (auto &lv : op->pre.levels) ps += int(lv.prog.launches.size());
    s->pre_stages = ps;
    s->build_seconds = op->build_seconds;
    s->precond_seconds = op->pre.seconds;
    s->id_count = op->id_count;
    s->io_rows_fwd = op->fwd.io_rows;
    s->precond_reconstructions = op->pre.reconstructions;
    s->precond_sketch_cols = op->pre.sketch_cols;
    s->io_rows_pre = op->pre.leaf.io_rows;
    for (auto &lv : op->pre.levels) s->io_rows_pre += lv.prog.io_rows;
  });
}

static void export_bytes(const void *src, size_t n, void *buf, size_t *bytes) {
  if (!buf) {
    *bytes = n;
    return;
  }
  if (*bytes < n) fail(HODBF_E_ARG, "export buffer too small");
  if (n) std::memcpy(buf, src, n);
  *bytes = n;
}

static float f16_to_f32(uint32_t h) {
  const uint32_t sign = (h & 0x8000u) << 16, e = (h >> 10) & 0x1F, m = h & 0x3FFu;
  uint32_t x;
  if (e == 0) {
    if (m == 0) x = sign;
    else {  // subnormal: value m * 2^-24
      float f = float(m) * 5.9604644775390625e-8f;
      std::memcpy(&x, &f, 4);
      x |= sign;
    }
  } else if (e == 31) {
    x = sign | 0x7F800000u | (m << 13);
  } else {
    x = sign | ((e - 15 + 127) << 23) | (m << 13);
  }
  float f;
  std::memcpy(&f, &x, 4);
  return f;
}

// ft: FT_C64 / FT_BF16 / FT_F16 storage; scales (per table row) restore block values.
static void export_arena(const DevBuf &a, int ft, const std::vector<BlockRec> *table,
                         const std::vector<float> *scales, void *buf, size_t *bytes) {
  const size_t count = ft == FT_C64 ? a.bytes / 8 : a.bytes / 4;
  const size_t need = count * sizeof(float) * 2;
  if (!buf) {
    *bytes = need;
    return;
  }
  if (*bytes < need) fail(HODBF_E_ARG, "export buffer too small");
  float *o = static_cast<float *>(buf);
  if (ft == FT_C64) {
    HIPCHK(hipMemcpy(buf, a.p, need, hipMemcpyDeviceToHost));
  } else {
    std::vector<uint32_t> tmp(count);
    HIPCHK(hipMemcpy(tmp.data(), a.p, count * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < count; ++i) {
      if (ft == FT_BF16) {
        uint32_t lo = (tmp[i] & 0xFFFFu) << 16, hi = tmp[i] & 0xFFFF0000u;
        std::memcpy(o + 2 * i, &lo, 4);
        std::memcpy(o + 2 * i + 1, &hi, 4);
      } else {
        o[2 * i] = f16_to_f32(tmp[i] & 0xFFFFu);
        o[2 * i + 1] = f16_to_f32(tmp[i] >> 16);
      }
    }
  }
  if (table && scales)
    for (size_t r = 0; r < table->size(); ++r) {
      const BlockRec &b = (*table)[r];
      const float s = (*scales)[r];
      for (int64_t k = 0; k < b.n; ++k)
        for (int64_t i = 0; i < b.m; ++i) {
          const int64_t e = b.off + k * b.lda + i;
          o[2 * e] *= s;
          o[2 * e + 1] *= s;
        }
    }
  *bytes = need;
}

hodbf_status hodbf_export(const hodbf_op *op, int32_t which, void *buf, size_t *bytes) {
  return guarded([&] {
    if (!op || !bytes) fail(HODBF_E_ARG, "NULL argument");
    switch (which) {
      case 0:
        export_bytes(op->tree.perm.data(), op->tree.perm.size() * 4, buf, bytes);
        break;
      case 1:
        export_bytes(op->fwd_table.data(), op->fwd_table.size() * sizeof(BlockRec), buf, bytes);
        break;
      case 2:
        export_arena(op->fwdF, FT_C64, nullptr, nullptr, buf, bytes);
        break;
      case 3:
        export_bytes(op->pre.table.data(), op->pre.table.size() * sizeof(BlockRec), buf, bytes);
        break;
      case 4:
      case 5:
      case 6: {
        const DevBuf &a = which == 4 ? op->pre.F32 : (which == 5 ? op->pre.BF16 : op->pre.F16);
        if (!a.p) fail(HODBF_E_STATE, "that preconditioner copy is not stored");
        export_arena(a, which == 4 ? FT_C64 : (which == 5 ? FT_BF16 : FT_F16), &op->pre.table,
                     &op->pre.scales, buf, bytes);
        break;
      }
      default:
        fail(HODBF_E_ARG, "unknown export selector");
    }
  });
}

// Host-only plan export (cached for the last parameter set).
static std::mutex g_probe_mu;
static std::vector<int32_t> g_probe_perm, g_probe_skel;
static std::vector<BlockRec> g_probe_table;
static std::vector<double> g_probe_vals;
static std::vector<double> g_probe_key;

hodbf_status hodbf_plan_probe(const hodbf_build_params *params, int32_t which, void *buf,
                              size_t *bytes) {
  return guarded([&] {
    if (!params || !bytes) fail(HODBF_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_probe_mu);
    const int64_t n = int64_t(params->nx) * params->ny * params->nz;
    std::vector<double> key = {double(params->nx), double(params->ny), double(params->nz),
                               params->h, params->k0, params->tol_con, double(params->leaf_size),
                               double(params->seed)};
    if (params->eps_r && n > 0 && n < (int64_t(1) << 28))
      key.insert(key.end(), params->eps_r, params->eps_r + 2 * n);
    if (key != g_probe_key) {
      FwdPlan fp = build_forward_plan(*params);
      g_probe_perm = fp.tree.perm;
      g_probe_table.clear();
      g_probe_vals.clear();
      g_probe_skel.clear();
      auto put = [&](const Mat &f) {
        const int64_t off = int64_t(g_probe_vals.size() / 2);
        for (auto &v : f.v) {
          g_probe_vals.push_back(v.real());
          g_probe_vals.push_back(v.imag());
        }
        return off;
      };
      for (auto &bf : fp.bfs) {
        for (int64_t b = 0; b < int64_t(bf.V0.size()); ++b) {
          const Mat &f = bf.V0[size_t(b)];
          g_probe_table.push_back({1, bf.hod_level, bf.oi, 0, 0, 0, 0, b, f.m, f.n, put(f), f.m});
        }
        for (int l = 1; l <= bf.L; ++l) {
          const int64_t nb = int64_t(1) << (bf.L - l);
          for (int64_t e = 0; e < int64_t(bf.W[l].size()); ++e) {
            const Mat &f = bf.W[l][size_t(e)];
            g_probe_table.push_back({2, bf.hod_level, bf.oi, 0, 0, l, e / nb, e % nb, f.m, f.n, put(f), f.m});
          }
        }
        for (int64_t a = 0; a < int64_t(bf.bskel.size()); ++a) {
          const auto &sk = bf.bskel[size_t(a)];
          g_probe_table.push_back({3, bf.hod_level, bf.oi, 0, 0, bf.L, a, 0, 0, int64_t(sk.size()),
                                   int64_t(g_probe_skel.size()), 0});
          g_probe_skel.insert(g_probe_skel.end(), sk.begin(), sk.end());
        }
      }
      g_probe_key = key;
    }
    switch (which) {
      case 0:
        export_bytes(g_probe_perm.data(), g_probe_perm.size() * 4, buf, bytes);
        break;
      case 1:
        export_bytes(g_probe_table.data(), g_probe_table.size() * sizeof(BlockRec), buf, bytes);
        break;
      case 2:
        export_bytes(g_probe_vals.data(), g_probe_vals.size() * 8, buf, bytes);
        break;
      case 6:
        export_bytes(g_probe_skel.data(), g_probe_skel.size() * 4, buf, bytes);
        break;
      default:
        fail(HODBF_E_ARG, "unknown probe selector");
    }
  });
}

}  // extern "C"
