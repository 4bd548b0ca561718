// vie_solve: right-preconditioned flexible GMRES(m) for Z x = b (eq. (4) / eq. (precon)),
// all Krylov arithmetic in complex FP64 on the device; products with Z and P run
// through the grouped-GEMM programs in complex FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <type_traits>
#include <vector>

#include "construct_dev.h"
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

// Arithmetic of the preconditioner products selected by use_precond (-1: none).
static int precond_ftype(const hodbf_op &op, int use_precond) {
  if (use_precond == 0) return -1;
  if (use_precond == 1) {
    if (!op.pre.present) fail(HODBF_E_STATE, "operator has no preconditioner");
    return op.pre.default_ft;
  }
  if (use_precond == 8 + HODBF_P_FP32) {
    if (!op.pre.F32.p) fail(HODBF_E_STATE, "no FP32 preconditioner copy");
    return FT_C64;
  }
  if (use_precond == 16 + HODBF_P_FP32) {
    if (!op.pre.F32.p) fail(HODBF_E_STATE, "no FP32 preconditioner copy");
    return FT_C64_S3;
  }
  if (use_precond == 8 + HODBF_P_BF16) {
    if (!op.pre.BF16.p) fail(HODBF_E_STATE, "no BF16 preconditioner copy");
    return FT_BF16;
  }
  if (use_precond == 8 + HODBF_P_FP16) {
    if (!op.pre.F16.p) fail(HODBF_E_STATE, "no FP16 preconditioner copy");
    return FT_F16;
  }
  fail(HODBF_E_ARG, "unknown use_precond");
}

// The last columns of a solve (at most kF64Cols still iterating) run their products
// with Z in FP64 arithmetic over the FP32-stored factors, inside the Arnoldi process and
// for the true residual.  Products that round their input and accumulate in FP32 err by
// about u32 ||Z|| ||z||; for a column whose Krylov vectors reach the ill-conditioned
// directions that P amplifies, that error approaches the residual still to be removed,
// and the column stalls just above tol, each restart undoing what the last one gained.
constexpr int kF64Cols = 16;

// y = Z_con x in FP64 (x, y tree order, R columns interleaved; T: stage workspace)
static void forward_f64(const hodbf_op &op, const double2 *x, double2 *T, double2 *y, int R,
                        hipStream_t st) {
  for (const Launch &ln : op.fwd.launches)
    launch_grouped_f64(op.fwd.segs.as<Seg>(), op.fwd.pairs.as<Pair>(), op.fwd.rowmap.as<RowMap>(),
                       ln.s0, ln.ns, op.fwdF.as<float2>(), x, T, ln.out ? y : T, R, ln.beta, st);
}

// Device workspace of one solve: every buffer solve_impl carves, each rounded up to 256
// bytes plus 256 of alignment slack.
static size_t solve_workspace(const hodbf_op &op, int R, int m, bool pre) {
  const int64_t n = op.n;
  const int64_t NR = n * R;
  const int nblk = multidot_blocks(n, R);
  const int64_t wrows = std::max(forward_work_rows(op), pre ? precond_work_rows(op) : 0);
  size_t need = 0;
  auto add = [&](size_t b) { need += ((b + 255) & ~size_t(255)) + 256; };
  add(NR * 16);                 // bt
  add(NR * 16);                 // xt
  add(NR * 16);                 // rt (residual of the last cycle, all columns)
  add(NR * 16);                 // xc (solution of the cycle's columns)
  add(size_t(std::max<int64_t>(n, int64_t(m + 1) * m)) * R * 16);  // column-gather staging
  add(size_t(R) * 4 * 2);                                           // column lists
  add(size_t(m + 1) * NR * 16); // V
  add(size_t(m) * NR * 8);      // Zs
  add(NR * 16);                 // w
  add(NR * 8);                  // wf
  add(NR * 8);                  // vf
  add(size_t(std::max<int64_t>(wrows, 1)) * R * 8);  // apply workspace
  add(size_t(std::max<int64_t>(forward_work_rows(op), 1)) * std::min(R, kF64Cols) * 16);  // FP64 apply workspace
  add(size_t(nblk) * (m + 1) * R * 16);             // partials
  add(size_t(m + 1) * m * R * 16);                  // H
  add(size_t(m) * R * 16 * 2);                      // cs, sn
  add(size_t(m + 1) * R * 16);                      // g
  add(size_t(m) * R * 16);                          // y
  add(size_t(m + 1) * R * 16);                      // hbuf
  add(size_t(R) * 16);                              // sq
  add(size_t(R) * 8 * 2);                           // bnorm, est
  add(size_t(R) * 4 * 2);                           // jend, active
  return need;
}

static void solve_impl(const hodbf_op &op, int R, const void *b, int64_t ldb, void *x,
                       int64_t ldx, const hodbf_solve_opts &o, hodbf_solve_info *info,
                       hipStream_t st, hodbf_status &status) {
  const int64_t n = op.n;
  const int m = o.restart;
  const int pre_ft = precond_ftype(op, o.use_precond);
  const int f64cols = o.fp32_only ? 0 : kF64Cols;
  const int64_t NR = n * R;
  const int nblk = multidot_blocks(n, R);
  const int64_t wrows = std::max(forward_work_rows(op), pre_ft >= 0 ? precond_work_rows(op) : 0);
  const size_t ws = solve_workspace(op, R, m, pre_ft >= 0);
  const Scratch scr(ws, st);
  Carve cv{scr.as<char>()};
  double2 *bt = cv.take<double2>(NR), *xt = cv.take<double2>(NR);
  double2 *rt = cv.take<double2>(NR), *xc = cv.take<double2>(NR);
  void *stage = cv.take<double2>(size_t(std::max<int64_t>(n, int64_t(m + 1) * m)) * R);
  int32_t *colidx = cv.take<int32_t>(R), *keepidx = cv.take<int32_t>(R);
  double2 *V = cv.take<double2>(size_t(m + 1) * NR);
  float2 *Zs = cv.take<float2>(size_t(m) * NR);
  double2 *w = cv.take<double2>(NR);
  float2 *wf = cv.take<float2>(NR), *vf = cv.take<float2>(NR);
  float2 *work = cv.take<float2>(size_t(std::max<int64_t>(wrows, 1)) * R);
  double2 *work64 = cv.take<double2>(size_t(std::max<int64_t>(forward_work_rows(op), 1)) *
                                     std::min(R, kF64Cols));
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
  if (cv.off > ws) fail(HODBF_E_HIP, "internal: solve buffers exceed the sized workspace");

  const int32_t *tpos = op.dev.tpos.as<int32_t>(), *perm = op.dev.perm.as<int32_t>();
  auto norms2 = [&](const double2 *v, std::vector<double> &out) {
    launch_multidot(v, 0, 1, v, n, R, partial, nblk, st);
    launch_reduce_partials(partial, nblk, 1, R, sq, 0, st);
    std::vector<double2> h(static_cast<size_t>(R));
    HIPCHK(hipMemcpyAsync(h.data(), sq, size_t(R) * 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out.resize(static_cast<size_t>(R));
    for (int q = 0; q < R; ++q) out[size_t(q)] = h[size_t(q)].x;
  };

  // Host-to-device copies of small host vectors: the source is kept alive until the solve
  // returns, so its lifetime never depends on when the asynchronous copy reads it.
  std::deque<std::vector<char>> held;
  // On every exit, normal or by error, the stream drains before `held` is released.
  struct DrainOnExit {
    hipStream_t st;
    ~DrainOnExit() { (void)hipStreamSynchronize(st); }
  } drain{st};
  auto upload = [&](void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return;
    held.emplace_back(static_cast<const char *>(src), static_cast<const char *>(src) + bytes);
    HIPCHK(hipMemcpyAsync(dst, held.back().data(), bytes, hipMemcpyHostToDevice, st));
  };
  // Gather the columns idx (device, Rd of them) of a [rows][Rs] block into a [rows][Rd]
  // block at dst (which may overlap src: the gather goes through the staging buffer).
  auto compact = [&](auto *src, auto *dst, int64_t rows, int Rs, const int32_t *idx, int Rd) {
    using T = std::remove_pointer_t<decltype(dst)>;
    T *tmp = static_cast<T *>(stage);
    launch_gather_cols<T>(src, rows, Rs, idx, Rd, tmp, st);
    if (rows * Rd > 0)
      HIPCHK(hipMemcpyAsync(dst, tmp, size_t(rows * Rd) * sizeof(T), hipMemcpyDeviceToDevice, st));
  };

  launch_gather(b, true, ldb, bt, true, tpos, n, R, st);
  HIPCHK(hipMemsetAsync(xt, 0, NR * 16, st));
  std::vector<double> bn2, rn2;
  norms2(bt, bn2);
  std::vector<double> bnorm(static_cast<size_t>(R)), relres(static_cast<size_t>(R), 0.0);
  std::vector<double> target(static_cast<size_t>(R), 1.0);
  std::vector<int32_t> active(static_cast<size_t>(R)), iters(static_cast<size_t>(R), 0);
  for (int q = 0; q < R; ++q) {
    bnorm[size_t(q)] = std::sqrt(bn2[size_t(q)]);
    if (!std::isfinite(bnorm[size_t(q)])) fail(HODBF_E_NUMERIC, "non-finite right-hand side");
    active[size_t(q)] = bnorm[size_t(q)] > 0 ? 1 : 0;
  }
  HIPCHK(hipMemcpyAsync(rt, bt, NR * 16, hipMemcpyDeviceToDevice, st));  // r0 = b (x0 = 0)
  int64_t steps = 0;
  bool numeric_bad = false;
  // Each restart cycle works on the columns still active, stored compactly (Rc columns,
  // cur[k] = original column of compact column k).  Columns whose estimated residual
  // meets the tolerance inside a cycle stop iterating; once enough of them have, they
  // take their least-squares update at once and every per-column array is compacted to
  // the columns still iterating, so later products run on fewer columns.  Every column
  // follows the same arithmetic as in a solve of its own.
  while (steps < o.max_iter && std::any_of(active.begin(), active.end(), [](int a) { return a; })) {
    std::vector<int32_t> act;
    for (int q = 0; q < R; ++q)
      if (active[size_t(q)]) act.push_back(q);
    const int Ra = int(act.size());
    std::vector<int32_t> cur = act;
    int Rc = Ra;
    upload(colidx, act.data(), size_t(Ra) * 4);
    launch_gather_cols<double2>(rt, n, R, colidx, Ra, w, st);
    launch_gather_cols<double2>(xt, n, R, colidx, Ra, xc, st);
    std::vector<double> bsub(static_cast<size_t>(Ra));
    // the Arnoldi estimate compares against tol times this norm: halved for a column
    // whose last cycle ended just above tol (see below)
    for (int k = 0; k < Ra; ++k)
      bsub[size_t(k)] = bnorm[size_t(act[size_t(k)])] * target[size_t(act[size_t(k)])];
    std::vector<int32_t> ones(static_cast<size_t>(Ra), 1);
    upload(gs.bnorm, bsub.data(), size_t(Ra) * 8);
    upload(gs.active, ones.data(), size_t(Ra) * 4);
    gs.R = Rc;
    launch_multidot(w, 0, 1, w, n, Rc, partial, nblk, st);
    launch_reduce_partials(partial, nblk, 1, Rc, sq, 0, st);
    launch_cycle_init(gs, sq, st);
    launch_normalize(w, sq, V, nullptr, n, Rc, nullptr, st);
    std::vector<int32_t> jend(static_cast<size_t>(Rc));
    // least-squares update x += Z_k y for the compact columns with jend >= 0 (the others
    // get y = 0), then their solutions go back to xt and their steps are counted
    auto finish = [&](int nv, const std::vector<int32_t> &jk) {
      std::vector<int32_t> jz(jk.size());
      for (size_t k = 0; k < jk.size(); ++k) jz[k] = jk[k] >= 0 ? jk[k] : 0;
      upload(gs.jend, jz.data(), jz.size() * 4);
      launch_lsq(gs, st);
      launch_xupdate(Zs, n * Rc, nv, gs.y, xc, n, Rc, st);
      for (size_t k = 0; k < jk.size(); ++k)
        if (jk[k] >= 0) iters[size_t(cur[k])] += jk[k];
    };
    int jdone = 0;
    const int jmax = int(std::min<int64_t>(m, o.max_iter - steps));
    for (int j = 0; j < jmax; ++j) {
      const int64_t NRc = n * Rc;
      double2 *vj = V + size_t(j) * NRc;
      float2 *zj = Zs + size_t(j) * NRc;
      launch_c128_to_c64(vj, vf, NRc, st);
      if (pre_ft >= 0) apply_precond_tree(op, pre_ft, vf, zj, work, Rc, st);
      else HIPCHK(hipMemcpyAsync(zj, vf, NRc * 8, hipMemcpyDeviceToDevice, st));
      if (Rc <= f64cols) {
        launch_c64_to_c128(zj, rt, NRc, st);  // rt is free until the cycle ends
        forward_f64(op, rt, work64, w, Rc, st);
      } else {
        apply_forward_tree(op, zj, wf, work, Rc, st);
        launch_c64_to_c128(wf, w, NRc, st);
      }
      double2 *hcol = gs.H + size_t(j) * (m + 1) * Rc;
      // classical Gram-Schmidt, applied twice
      launch_multidot(V, NRc, j + 1, w, n, Rc, partial, nblk, st);
      launch_reduce_partials(partial, nblk, j + 1, Rc, hcol, 0, st);
      launch_vupdate(V, NRc, j + 1, hcol, w, n, Rc, st);
      launch_multidot(V, NRc, j + 1, w, n, Rc, partial, nblk, st);
      launch_reduce_partials(partial, nblk, j + 1, Rc, hbuf, 0, st);
      launch_vupdate(V, NRc, j + 1, hbuf, w, n, Rc, st);
      launch_reduce_partials(partial, nblk, j + 1, Rc, hcol, 1, st);
      launch_multidot(w, 0, 1, w, n, Rc, partial, nblk, st);
      launch_reduce_partials(partial, nblk, 1, Rc, sq, 0, st);
      launch_normalize(w, sq, V + size_t(j + 1) * NRc, hcol + size_t(j + 1) * Rc, n, Rc, nullptr,
                       st);
      launch_givens(gs, j, o.tol, st);
      HIPCHK(hipGetLastError());
      jend.resize(size_t(Rc));
      HIPCHK(hipMemcpyAsync(jend.data(), gs.jend, size_t(Rc) * 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      jdone = j + 1;
      std::vector<int32_t> keep;
      for (int k = 0; k < Rc; ++k)
        if (jend[size_t(k)] < 0) keep.push_back(k);
      if (keep.empty()) break;
      const int done = Rc - int(keep.size());
      if (j + 1 < jmax && done >= std::max(4, Rc / 8)) {
        // retire the finished columns, then compact to the columns still iterating
        finish(jdone, jend);
        std::vector<int32_t> fin;
        for (int k = 0; k < Rc; ++k)
          if (jend[size_t(k)] >= 0) fin.push_back(k);
        std::vector<int32_t> fin_orig;
        for (int k : fin) fin_orig.push_back(cur[size_t(k)]);
        upload(keepidx, fin.data(), fin.size() * 4);
        upload(colidx, fin_orig.data(), fin_orig.size() * 4);
        double2 *tmp = static_cast<double2 *>(stage);
        launch_gather_cols<double2>(xc, n, Rc, keepidx, int(fin.size()), tmp, st);
        launch_scatter_cols<double2>(tmp, n, int(fin.size()), colidx, R, xt, st);
        const int Rk = int(keep.size());
        upload(keepidx, keep.data(), size_t(Rk) * 4);
        for (int i = 0; i <= jdone; ++i)
          compact(V + size_t(i) * NRc, V + size_t(i) * n * Rk, n, Rc, keepidx, Rk);
        for (int i = 0; i < jdone; ++i)
          compact(Zs + size_t(i) * NRc, Zs + size_t(i) * n * Rk, n, Rc, keepidx, Rk);
        compact(xc, xc, n, Rc, keepidx, Rk);
        compact(gs.H, gs.H, int64_t(m + 1) * m, Rc, keepidx, Rk);
        compact(gs.cs, gs.cs, int64_t(m), Rc, keepidx, Rk);
        compact(gs.sn, gs.sn, int64_t(m), Rc, keepidx, Rk);
        compact(gs.g, gs.g, int64_t(m + 1), Rc, keepidx, Rk);
        compact(gs.bnorm, gs.bnorm, 1, Rc, keepidx, Rk);
        compact(gs.est, gs.est, 1, Rc, keepidx, Rk);
        compact(gs.active, gs.active, 1, Rc, keepidx, Rk);
        // the kept columns are still iterating (finish() left 0 in their jend)
        const std::vector<int32_t> still(static_cast<size_t>(Rk), -1);
        upload(gs.jend, still.data(), size_t(Rk) * 4);
        std::vector<int32_t> nc;
        for (int k : keep) nc.push_back(cur[size_t(k)]);
        cur = nc;
        Rc = Rk;
        gs.R = Rc;
      }
    }
    // columns still iterating at the cycle cap keep all jdone steps
    for (int k = 0; k < Rc; ++k)
      if (jend[size_t(k)] < 0) jend[size_t(k)] = jdone;
    finish(jdone, jend);
    upload(colidx, cur.data(), size_t(Rc) * 4);
    launch_scatter_cols<double2>(xc, n, Rc, colidx, R, xt, st);
    steps += jdone;
    // true residual r = b - Z x for every column of this cycle
    upload(colidx, act.data(), size_t(Ra) * 4);
    launch_gather_cols<double2>(xt, n, R, colidx, Ra, xc, st);
    if (Ra <= f64cols) {
      forward_f64(op, xc, work64, w, Ra, st);
    } else {
      launch_c128_to_c64(xc, vf, n * Ra, st);
      apply_forward_tree(op, vf, wf, work, Ra, st);
      launch_c64_to_c128(wf, w, n * Ra, st);
    }
    launch_gather_cols<double2>(bt, n, R, colidx, Ra, xc, st);
    launch_axpby(xc, w, w, n * Ra, st);
    launch_scatter_cols<double2>(w, n, Ra, colidx, R, rt, st);
    launch_multidot(w, 0, 1, w, n, Ra, partial, nblk, st);
    launch_reduce_partials(partial, nblk, 1, Ra, sq, 0, st);
    std::vector<double2> h(static_cast<size_t>(Ra));
    HIPCHK(hipMemcpyAsync(h.data(), sq, size_t(Ra) * 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < Ra; ++k) {
      const int q = act[size_t(k)];
      const double rr = std::sqrt(h[size_t(k)].x) / bnorm[size_t(q)];
      relres[size_t(q)] = rr;
      // a cycle that met tol on its Arnoldi estimate but left the true residual just
      // above it fell into the gap FP32 products open between the two: the column's next
      // cycle aims at tol / 2, or it would stop again after a step or two that barely
      // move the true residual
      target[size_t(q)] = (rr > o.tol && rr <= 3 * o.tol) ? 0.5 : 1.0;
      if (!std::isfinite(rr)) {
        numeric_bad = true;
        active[size_t(q)] = 0;
      } else if (rr <= o.tol) {
        active[size_t(q)] = 0;
      }
    }
    if (numeric_bad) break;
    {
      double worst = 0;
      for (int k = 0; k < Ra; ++k) worst = std::max(worst, relres[size_t(act[size_t(k)])]);
      logf("fgmres: %d steps, %d of %d columns still active, worst true residual %.3e", steps,
           int(std::count(active.begin(), active.end(), 1)), R, worst);
    }
  }
  launch_scatter(xt, true, x, true, ldx, perm, n, R, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
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

static void check_solve_args(const hodbf_op *op, int32_t nrhs, const hodbf_solve_opts *opts) {
  if (!op || !opts) fail(HODBF_E_ARG, "NULL argument");
  if (nrhs < 0) fail(HODBF_E_ARG, "nrhs < 0");
  if (!(opts->tol > 0) || opts->restart < 1 || opts->restart > 200 || opts->max_iter < 1 ||
      (opts->fp32_only != 0 && opts->fp32_only != 1))
    fail(HODBF_E_ARG, "bad solve options");
}

extern "C" hodbf_status hodbf_solve_workspace(const hodbf_op *op, int32_t nrhs,
                                              const hodbf_solve_opts *opts, size_t *bytes) {
  try {
    if (!bytes) fail(HODBF_E_ARG, "NULL argument");
    check_solve_args(op, nrhs, opts);
    const int pre_ft = precond_ftype(*op, opts->use_precond);
    *bytes = nrhs == 0 ? 0 : solve_workspace(*op, nrhs, opts->restart, pre_ft >= 0);
    return HODBF_OK;
  } catch (const Error &e) {
    set_last_error(e.msg);
    return e.code;
  } catch (...) {
    set_last_error("internal error in hodbf_solve_workspace");
    return HODBF_E_HIP;
  }
}

extern "C" hodbf_status vie_solve(const hodbf_op *op, int32_t nrhs, const void *b, int64_t ldb,
                                  void *x, int64_t ldx, const hodbf_solve_opts *opts,
                                  hodbf_solve_info *info, void *stream) {
  hodbf_status result = HODBF_OK;
  try {
    check_solve_args(op, nrhs, opts);
    if (nrhs == 0) return HODBF_OK;
    if (!b || !x || ldb < op->n || ldx < op->n) fail(HODBF_E_ARG, "bad b / x / leading dimension");
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
