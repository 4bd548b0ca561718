// vie_solve: right-preconditioned flexible GMRES(m) for Z x = b (eq. (4) / eq. (precon)),
// all Krylov arithmetic in complex FP64 on the device; products with Z and P run
// through the grouped-GEMM programs in complex FP32.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "op.h"

namespace hodbf {


namespace {

struct Carve {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace

static void solve_impl(const hodbf_op &op, int R, const void *b, int64_t ldb, void *x,
                       int64_t ldx, const hodbf_solve_opts &o, hodbf_solve_info *info,
                       hipStream_t st, hodbf_status &status) {
  const int64_t n = op.n;
  const int m = o.restart;
  int pre_ft = -1;
  if (o.use_precond == 1) {
    if (!op.pre.present) fail(HODBF_E_STATE, "operator has no preconditioner");
    pre_ft = op.pre.default_ft;
  } else if (o.use_precond == 8 + HODBF_P_FP32) {
    if (!op.pre.F32.p) fail(HODBF_E_STATE, "no FP32 preconditioner copy");
    pre_ft = FT_C64;
  } else if (o.use_precond == 8 + HODBF_P_BF16) {
    if (!op.pre.BF16.p) fail(HODBF_E_STATE, "no BF16 preconditioner copy");
    pre_ft = FT_BF16;
  } else if (o.use_precond == 8 + HODBF_P_FP16) {
    if (!op.pre.F16.p) fail(HODBF_E_STATE, "no FP16 preconditioner copy");
    pre_ft = FT_F16;
  } else if (o.use_precond != 0) {
    fail(HODBF_E_ARG, "unknown use_precond");
  }
  const int64_t NR = n * R;
  const int nblk = multidot_blocks(n, R);
  const int64_t wrows = std::max(forward_work_rows(op), pre_ft >= 0 ? precond_work_rows(op) : 0);
  // workspace sizing (bytes, with alignment slack)
  size_t need = 0;
  auto add = [&](size_t b) { need += ((b + 255) & ~size_t(255)) + 256; };
  add(NR * 16);                 // bt
  add(NR * 16);                 // xt
  add(size_t(m + 1) * NR * 16); // V
  add(size_t(m) * NR * 8);      // Zs
  add(NR * 16);                 // w
  add(NR * 8);                  // wf
  add(NR * 8);                  // vf
  add(size_t(std::max<int64_t>(wrows, 1)) * R * 8);  // apply workspace
  add(size_t(nblk) * (m + 1) * R * 16);             // partials
  add(size_t(m + 1) * m * R * 16);                  // H
  add(size_t(m) * R * 16 * 2);                      // cs, sn
  add(size_t(m + 1) * R * 16);                      // g
  add(size_t(m) * R * 16);                          // y
  add(size_t(m + 1) * R * 16);                      // hbuf
  add(size_t(R) * 16);                              // sq
  add(size_t(R) * 8 * 2);                           // bnorm, est
  add(size_t(R) * 4 * 2);                           // jend, active
  char *base = static_cast<char *>(scratch_alloc(need, st));
  Carve cv{base};
  double2 *bt = cv.take<double2>(NR), *xt = cv.take<double2>(NR);
  double2 *V = cv.take<double2>(size_t(m + 1) * NR);
  float2 *Zs = cv.take<float2>(size_t(m) * NR);
  double2 *w = cv.take<double2>(NR);
  float2 *wf = cv.take<float2>(NR), *vf = cv.take<float2>(NR);
  float2 *work = cv.take<float2>(size_t(std::max<int64_t>(wrows, 1)) * R);
  double2 *partial = cv.take<double2>(size_t(nblk) * (m + 1) * R);
  GmresState gs;
  gs.m = m;
  gs.R = R;
  gs.H = cv.take<double2>(size_t(m + 1) * m * R);
  gs.cs = cv.take<double2>(size_t(m) * R);
  gs.sn = cv.take<double2>(size_t(m) * R);
  gs.g = cv.take<double2>(size_t(m + 1) * R);
  gs.y = cv.take<double2>(size_t(m) * R);
  double2 *hbuf = cv.take<double2>(size_t(m + 1) * R);
  double2 *sq = cv.take<double2>(R);
  gs.bnorm = cv.take<double>(R);
  gs.est = cv.take<double>(R);
  gs.jend = cv.take<int32_t>(R);
  gs.active = cv.take<int32_t>(R);

  const int32_t *perm = op.dev.perm.as<int32_t>();
  auto norms2 = [&](const double2 *v, std::vector<double> &out) {
    launch_multidot(v, 0, 1, v, n, R, partial, nblk, st);
    launch_reduce_partials(partial, nblk, 1, R, sq, 0, st);
    std::vector<double2> h(static_cast<size_t>(R));
    HIPCHK(hipMemcpyAsync(h.data(), sq, size_t(R) * 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out.resize(static_cast<size_t>(R));
    for (int q = 0; q < R; ++q) out[size_t(q)] = h[size_t(q)].x;
  };
  auto applyZ = [&](const float2 *in, double2 *out) {
    apply_forward_tree(op, in, wf, work, R, st);
    launch_c64_to_c128(wf, out, NR, st);
  };

  launch_gather(b, true, ldb, bt, true, perm, n, R, st);
  HIPCHK(hipMemsetAsync(xt, 0, NR * 16, st));
  std::vector<double> bn2, rn2;
  norms2(bt, bn2);
  std::vector<double> bnorm(static_cast<size_t>(R)), relres(static_cast<size_t>(R), 0.0);
  std::vector<int32_t> active(static_cast<size_t>(R)), iters(static_cast<size_t>(R), 0), jend(static_cast<size_t>(R));
  for (int q = 0; q < R; ++q) {
    bnorm[size_t(q)] = std::sqrt(bn2[size_t(q)]);
    if (!std::isfinite(bnorm[size_t(q)])) fail(HODBF_E_NUMERIC, "non-finite right-hand side");
    active[size_t(q)] = bnorm[size_t(q)] > 0 ? 1 : 0;
  }
  HIPCHK(hipMemcpyAsync(gs.bnorm, bnorm.data(), size_t(R) * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w, bt, NR * 16, hipMemcpyDeviceToDevice, st));  // r0 = b (x0 = 0)
  int64_t steps = 0;
  bool numeric_bad = false;
  while (steps < o.max_iter && std::any_of(active.begin(), active.end(), [](int a) { return a; })) {
    HIPCHK(hipMemcpyAsync(gs.active, active.data(), size_t(R) * 4, hipMemcpyHostToDevice, st));
    launch_multidot(w, 0, 1, w, n, R, partial, nblk, st);
    launch_reduce_partials(partial, nblk, 1, R, sq, 0, st);
    launch_cycle_init(gs, sq, st);
    launch_normalize(w, sq, V, nullptr, n, R, nullptr, st);
    launch_mask_cols(V, gs.active, n, R, st);
    int jdone = 0;
    const int jmax = int(std::min<int64_t>(m, o.max_iter - steps));
    for (int j = 0; j < jmax; ++j) {
      double2 *vj = V + size_t(j) * NR;
      float2 *zj = Zs + size_t(j) * NR;
      launch_c128_to_c64(vj, vf, NR, st);
      if (pre_ft >= 0) apply_precond_tree(op, pre_ft, vf, zj, work, R, st);
      else HIPCHK(hipMemcpyAsync(zj, vf, NR * 8, hipMemcpyDeviceToDevice, st));
      applyZ(zj, w);
      double2 *hcol = gs.H + size_t(j) * (m + 1) * R;
      // classical Gram-Schmidt, applied twice
      launch_multidot(V, NR, j + 1, w, n, R, partial, nblk, st);
      launch_reduce_partials(partial, nblk, j + 1, R, hcol, 0, st);
      launch_vupdate(V, NR, j + 1, hcol, w, n, R, st);
      launch_multidot(V, NR, j + 1, w, n, R, partial, nblk, st);
      launch_reduce_partials(partial, nblk, j + 1, R, hbuf, 0, st);
      launch_vupdate(V, NR, j + 1, hbuf, w, n, R, st);
      launch_reduce_partials(partial, nblk, j + 1, R, hcol, 1, st);
      launch_multidot(w, 0, 1, w, n, R, partial, nblk, st);
      launch_reduce_partials(partial, nblk, 1, R, sq, 0, st);
      launch_normalize(w, sq, V + size_t(j + 1) * NR, hcol + size_t(j + 1) * R, n, R, nullptr, st);
      launch_givens(gs, j, o.tol, st);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(jend.data(), gs.jend, size_t(R) * 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      jdone = j + 1;
      bool all = true;
      for (int q = 0; q < R; ++q)
        if (jend[size_t(q)] < 0) all = false;
      if (all) break;
    }
    // columns still iterating at the cycle cap keep all jdone steps
    for (int q = 0; q < R; ++q)
      if (jend[size_t(q)] < 0) jend[size_t(q)] = jdone;
    HIPCHK(hipMemcpyAsync(gs.jend, jend.data(), size_t(R) * 4, hipMemcpyHostToDevice, st));
    launch_lsq(gs, st);
    launch_xupdate(Zs, NR, jdone, gs.y, xt, n, R, st);
    for (int q = 0; q < R; ++q)
      if (active[size_t(q)]) iters[size_t(q)] += jend[size_t(q)];
    steps += jdone;
    // true residual r = b - Z x
    launch_c128_to_c64(xt, vf, NR, st);
    applyZ(vf, w);
    launch_axpby(bt, w, w, NR, st);
    norms2(w, rn2);
    for (int q = 0; q < R; ++q) {
      if (!active[size_t(q)]) continue;
      const double rr = std::sqrt(rn2[size_t(q)]) / bnorm[size_t(q)];
      relres[size_t(q)] = rr;
      if (!std::isfinite(rr)) {
        numeric_bad = true;
        active[size_t(q)] = 0;
      } else if (rr <= o.tol) {
        active[size_t(q)] = 0;
      }
    }
    if (numeric_bad) break;
  }
  launch_scatter(xt, true, x, true, ldx, perm, n, R, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  scratch_free(base, st);
  bool allconv = true;
  for (int q = 0; q < R; ++q) {
    const bool c = bnorm[size_t(q)] == 0 || relres[size_t(q)] <= o.tol;
    allconv = allconv && c;
    if (info) {
      if (info->iters) info->iters[q] = iters[size_t(q)];
      if (info->converged) info->converged[q] = c ? 1 : 0;
      if (info->relres) info->relres[q] = relres[size_t(q)];
    }
  }
  if (numeric_bad) fail(HODBF_E_NUMERIC, "non-finite residual");
  status = allconv ? HODBF_OK : HODBF_E_NOCONV;
}

}  // namespace hodbf

using namespace hodbf;

extern "C" hodbf_status vie_solve(const hodbf_op *op, int32_t nrhs, const void *b, int64_t ldb,
                                  void *x, int64_t ldx, const hodbf_solve_opts *opts,
                                  hodbf_solve_info *info, void *stream) {
  hodbf_status result = HODBF_OK;
  try {
    if (!op || !opts) fail(HODBF_E_ARG, "NULL argument");
    if (nrhs < 0) fail(HODBF_E_ARG, "nrhs < 0");
    if (nrhs == 0) return HODBF_OK;
    if (!b || !x || ldb < op->n || ldx < op->n) fail(HODBF_E_ARG, "bad b / x / leading dimension");
    if (!(opts->tol > 0) || opts->restart < 1 || opts->restart > 200 || opts->max_iter < 1)
      fail(HODBF_E_ARG, "bad solve options");
    solve_impl(*op, nrhs, b, ldb, x, ldx, *opts, info, static_cast<hipStream_t>(stream), result);
    if (result == HODBF_E_NOCONV) set_last_error("GMRES reached max_iter before tol");
    return result;
  } catch (const Error &e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return HODBF_E_NOMEM;
  } catch (...) {
    set_last_error("internal error in vie_solve");
    return HODBF_E_HIP;
  }
}
