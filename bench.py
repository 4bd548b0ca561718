#!/usr/bin/env python3
"""Benchmark of the HOD-BF VIE hot path on one MI355X.

One step = one preconditioned FGMRES solve of the whole right-hand-side batch to
chi_sol: FP32 forward HOD-BF apply, the preconditioner's FP32-stored factors on
split-BF16 MFMA with FP32 accumulation, FP64 Krylov arithmetic, 64 right-hand sides
batched.  The workload is 32^3 = 32768 voxels in a 4-wavelength cube, eps_r i.i.d.
U[2, 10], 64 seeded plane waves, leaf 64, chi_con 1e-4, chi_sol 1e-4; the preconditioner
is Algorithm 1 built on the device (BF_SMW with randomized butterfly reconstruction)
at chi_fact 1e-5 from exact dense inverses of the 1024-unknown nodes.

Also measured (inputs resident in HBM, HIP events on the launch stream):
  * the forward apply alone: GFLOP/s = 8 * R * (stored complex entries) / time;
  * the plain form: FP32 everything, one right-hand side at a time;
  * the same batched solve with the FP32, FP16 and BF16 arithmetic of the preconditioner;
  * the oracle on the host CPU (a bounded sample of FGMRES steps, see cpu_baseline), with
    all host cores allowed and with one.
``--mode apply`` runs applies only (and one device copy of known size, the reference
for traffic counters); it is the profiled command.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "c2_batched_32"
TOL_SOL = 1e-4
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_BF16_MFMA_TFLOPS = 2500.0
# HBM bytes of one apply of this workload (R = 64) per kernel, from the FETCH_SIZE /
# WRITE_SIZE counter runs recorded in profiles/*_traffic.md (FETCH_SIZE scaled by what
# it reads for a 256 MiB device copy, 131,083.5 KiB; WRITE_SIZE reads that copy as
# 262,144 KiB); valid only while the kernel and packing sources hash to sources_sha256.
MEASURED_TRAFFIC = {"sources_sha256": "189b6a0e73b6b871e55f5c316a9955663b659415f8f11ee0441f11cbee528684",
                    "precond_s3": {"bytes_per_apply": 5490977272.4 + 1292105616.0,
                                   "launches_per_apply": 41},
                    "forward_f32": {"bytes_per_apply": 1312039988.2 + 438161904.0,
                                    "launches_per_apply": 10},
                    "forward_s3": {"bytes_per_apply": None, "launches_per_apply": 10}}


def measured_copy_gbs(nbytes=1 << 30, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second), the STREAM-like
    reference beside the 8 TB/s specification."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * nbytes / t / 1e9


def stage_roofline(op, st, R, t_fwd):
    """Roofline summed over the forward apply's stages from the real block dimensions:
    T_roof = sum_s max(F_s / F_peak, B_s / BW), F_s = 8 R sum m n, B_s = 8 sum m n +
    8 R (output rows + distinct input rows of the stage).  Stage 0 holds the V0 blocks
    (each column leaf read once), stage s the level-s transfer blocks (sibling blocks share
    their input), the last stage the dense leaf blocks and the outer blocks (output: every
    row once)."""
    tab = op.export(1, np.int64).reshape(-1, 12)
    kind, l, oi, lev, a, b, m, n = (tab[:, 0], tab[:, 1], tab[:, 2], tab[:, 5], tab[:, 6],
                                    tab[:, 7], tab[:, 8], tab[:, 9])
    stages = []
    sel = kind == 1
    stages.append(("V0", sel, float((m[sel]).sum()), float(st["n"])))
    for s in range(1, int(lev[kind == 2].max(initial=0)) + 1):
        sel = (kind == 2) & (lev == s)
        keys = {}
        for li, oii, ai, bi, ni in zip(l[sel], oi[sel], a[sel], b[sel], n[sel]):
            keys[(int(li), int(oii), int(ai) >> 1, int(bi))] = int(ni)
        stages.append((f"W{s}", sel, float(m[sel].sum()), float(sum(keys.values()))))
    sel = (kind == 0) | (kind == 3)
    stages.append(("final", sel, float(st["n"]), float(n[sel].sum())))
    f_peak = PEAK_FP32_MFMA_TFLOPS * 1e12
    bw = PEAK_HBM_GBS * 1e9
    t_roof, rows = 0.0, []
    for name, sel, out_rows, in_rows in stages:
        ent = float((m[sel] * n[sel]).sum())
        f = 8.0 * R * ent
        by = 8.0 * ent + 8.0 * R * (out_rows + in_rows)
        t = max(f / f_peak, by / bw)
        t_roof += t
        rows.append({"stage": name, "gflop": f / 1e9, "mbytes": by / 1e6,
                     "bound": "mfma" if f / f_peak >= by / bw else "hbm", "t_roof_us": t * 1e6})
    return {"t_roof_ms": t_roof * 1e3, "t_measured_ms": t_fwd * 1e3, "frac": t_roof / t_fwd,
            "stages": rows}


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "pack.cpp", "pack_sink.h"):
        with open(os.path.join(ROOT, "paper_2111_01730_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def precond_block_sums(op, R):
    """Sum of m n and of (m + n) R over the stored preconditioner blocks (exported table):
    the per-block factor and vector counts before any sharing of input rows."""
    tab = op.export(3, np.int64).reshape(-1, 12)
    m, n = tab[:, 8].astype(np.float64), tab[:, 9].astype(np.float64)
    return {"sum_mn": float((m * n).sum()), "sum_m_plus_n_R": float(((m + n) * R).sum()),
            "blocks": int(tab.shape[0])}


def c3_forward(Operator, P_NONE, reps: int) -> dict:
    """The forward apply of the 64^3 sphere (262,144 unknowns, 32 plane waves, chi_con
    1e-4) on the tree-order entry, HIP events on the launch stream."""
    import torch
    from synth import config
    cfg = config("c3_sphere_64")
    t0 = time.perf_counter()
    op = Operator(cfg["grid"], tol_con=cfg["tol"], seed=cfg["seed"])
    build = time.perf_counter() - t0
    st = op.stats()
    b = op.plane_wave(cfg["dirs"])
    perm = torch.as_tensor(op.perm().astype(np.int64), device="cuda")
    xt = b[perm].to(torch.complex64).contiguous()
    R = xt.shape[1]
    for _ in range(2):
        op.apply_tree(xt, 0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        op.apply_tree(xt, 0)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    fl = 8.0 * R * st["entries_fwd"]
    out = {"n": op.n, "nrhs": R, "build_s": build, "entries_fwd": st["entries_fwd"],
           "apply_ms": t * 1e3, "apply_gflops": fl / t / 1e9,
           "mfma_frac": fl / t / 1e12 / PEAK_FP32_MFMA_TFLOPS}
    op.close()
    return out


def cpu_baseline_leg(seconds: float, workload: str) -> dict:
    """The oracle timed on the host over a bounded sample of the workload: its own
    FGMRES(20) (complex FP64, no preconditioner: the oracle's multiplicative inverse is a
    dense construction, out of reach at this size) with its FFT-exact product on the first
    plane wave, for about ``seconds``.  If the run does not reach the tolerance, the
    steps it would need are projected from its own residual history (the log-linear
    trend of the estimated residual over the last restart cycles)."""
    from oracle import gmres, vie
    from synth import config
    cfg = config(workload)
    g = cfg["grid"]
    b = vie.plane_wave(g, cfg["dirs"][:1])[:, 0]

    def run(k):
        t0, c0 = time.perf_counter(), time.process_time()
        _, it, conv, hist = gmres.fgmres(lambda v: vie.fft_matvec(g, v), b, None, tol=TOL_SOL,
                                         restart=20, max_iter=k)
        return time.perf_counter() - t0, it, conv, hist, time.process_time() - c0

    t5 = run(5)[0]
    k = max(40, int(seconds / (t5 / 5)))
    t, it, conv, hist, cpu_s = run(k)
    sec_per_step = t / max(it, 1)
    if conv:
        steps = float(it)
    else:
        tail = np.log10(np.maximum(np.asarray(hist[len(hist) // 2:], dtype=float), 1e-300))
        slope = np.polyfit(np.arange(len(tail)), tail, 1)[0] if len(tail) >= 4 else 0.0
        steps = (it + (np.log10(TOL_SOL) - tail[-1]) / slope) if slope < 0 else float("inf")
    return dict(seconds=t, cpu_seconds=cpu_s, threads_busy=cpu_s / t, host_cpus=os.cpu_count(),
                steps_run=it, converged=bool(conv), residual=float(hist[-1]) if hist else 1.0,
                sec_per_step=sec_per_step, projected_steps=steps,
                solves_per_s=(1.0 / (sec_per_step * steps)) if np.isfinite(steps) else 0.0)


def oracle_mode(args) -> dict:
    """Times of the oracle (plain numpy/scipy FP64, not a tuned CPU library) on the host:
    16^3: dense Z, dense product, LU solve, unpreconditioned FGMRES to 1e-6, HOD-BF build
    (full-row interpolative decompositions, chi 1e-4) and apply; 32^3, 64^3, 128^3:
    direct-sum rows per second and the FFT-exact product.  Threads: whatever
    OMP_NUM_THREADS / the BLAS allow (run once with all cores and once with one)."""
    import platform
    from oracle import butterfly, gmres, vie
    from synth import config

    def best(fn, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return min(ts)

    out = {"mode": "oracle", "threads": os.environ.get("OMP_NUM_THREADS", "unset"),
           "cpu": platform.processor() or platform.machine(), "host_cpus": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    out["cpu"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    c1 = config("c1_plain_16")
    g = c1["grid"]
    b = vie.plane_wave(g, c1["dirs"])[:, 0]
    t0 = time.perf_counter()
    Z = vie.dense(g)
    r = {"n": g.n, "dense_build_s": time.perf_counter() - t0}
    log(f"[oracle] c1 dense Z built in {r['dense_build_s']:.1f} s")
    r["dense_matvec_s"] = best(lambda: Z @ b, 5)
    r["lu_solve_s"] = best(lambda: gmres.lu_solve(Z, b), 2)
    log(f"[oracle] c1 LU solve {r['lu_solve_s']:.2f} s")
    t0 = time.perf_counter()
    _, it, conv, _ = gmres.fgmres(lambda v: Z @ v, b, None, tol=1e-6)
    r.update(fgmres_s=time.perf_counter() - t0, fgmres_iters=it, fgmres_converged=bool(conv))
    log(f"[oracle] c1 FGMRES {r['fgmres_s']:.2f} s, {it} steps")
    t0 = time.perf_counter()
    H = butterfly.build_hodbf(g, 1e-4)
    r["hodbf_build_s"] = time.perf_counter() - t0
    r["hodbf_apply_s"] = best(lambda: H.apply(b), 3)
    out["c1_plain_16"] = r
    for name, nrows in (("c2_batched_32", 32), ("c3_sphere_64", 16), ("c5_slabs_128", 4)):
        cfg = config(name, sample_rows=nrows)
        g = cfg["grid"]
        x = vie.plane_wave(g, cfg["dirs"][:1])[:, 0]
        t_rows = best(lambda: vie.direct_rows(g, x, cfg["rows"]), 1)
        t_fft = best(lambda: vie.fft_matvec(g, x), 1)
        out[name] = {"n": g.n, "direct_rows_per_s": nrows / t_rows, "fft_matvec_s": t_fft}
        log(f"[oracle] {name}: {out[name]}")
    return out


def apply_mode(args, cfg, Operator, P_NONE):
    """Applies only (--which 0: the forward operator; 6: the preconditioner's FP32 copy on
    split-BF16 arithmetic, the mixed solve's form): one device copy of known size, then
    applies."""
    import numpy as np
    import torch

    from paper_2111_01730_amd.hodbf import P_FP32
    g = cfg["grid"]
    which = args.which
    if which not in (0, 2, 5, 6):
        raise SystemExit("--which must be 0, 2, 5 or 6")
    pre = which in (2, 6)
    op = Operator(g, tol_con=cfg["tol"], tol_fact=args.tol_fact if pre else 0.0,
                  precond=P_FP32 if pre else P_NONE, seed=cfg["seed"],
                  precond_dense_levels=args.precond_dense_levels if pre else 0)
    st = op.stats()
    dirs = np.asarray(cfg["dirs"])[: args.apply_nrhs or None]
    R = len(dirs)
    b = op.plane_wave(dirs)
    perm = torch.as_tensor(op.perm().astype(np.int64), device="cuda")
    xt = b[perm].to(torch.complex64).contiguous()
    ref = torch.empty(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB copy reference
    dst = torch.empty_like(ref)
    for _ in range(3):
        dst.copy_(ref)
    torch.cuda.synchronize()
    reps = max(1, args.steps)
    if args.user_order and which != 0:
        raise SystemExit("--user-order applies the forward operator (which 0)")
    # user order: the C ABI's hodbf_apply on complex FP64 columns (gather to tree order
    # and FP32, the apply, scatter back to user order and FP64)
    run = (lambda: op.apply(b)) if args.user_order else (lambda: op.apply_tree(xt, which))
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    ent = st["entries_pre"] if pre else st["entries_fwd"]
    fl = 8.0 * R * ent
    print(json.dumps({"mode": "apply", "which": which, "user_order": args.user_order,
                      "nrhs": R, "apply_ms": t * 1e3,
                      "apply_gflops": fl / t / 1e9,
                      "launches_per_apply": st["pre_stages"] if pre else st["fwd_stages"],
                      "entries": ent, "io_rows": st["io_rows_pre"] if pre else st["io_rows_fwd"],
                      "reps": reps, "copy_bytes": ref.numel() * 4}), flush=True)
    return 0


def solves_mode(args, cfg, Operator):
    """Only the batched mixed solves of the main measurement (the profiled command for the
    solve's kernel breakdown): --warmup untimed solves, then --steps timed ones."""
    import torch

    from paper_2111_01730_amd.hodbf import P_FP32
    op = Operator(cfg["grid"], tol_con=cfg["tol"], tol_fact=args.tol_fact, precond=P_FP32,
                  seed=cfg["seed"], precond_dense_levels=args.precond_dense_levels)
    b = op.plane_wave(cfg["dirs"])
    for _ in range(args.warmup):
        op.solve(b, tol=TOL_SOL, use_precond="fp32_split")
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(max(1, args.steps)):
        _, info = op.solve(b, tol=TOL_SOL, use_precond="fp32_split")
    torch.cuda.synchronize()
    t = (time.perf_counter() - ts) / max(1, args.steps)
    sums = precond_block_sums(op, int(b.shape[1]))
    print(json.dumps({"mode": "solves", "ms_per_solve": t * 1e3, "nrhs": int(b.shape[1]),
                      "precond_blocks": sums,
                      "iters_max": int(info["iters"].max()),
                      "iters_mean": float(info["iters"].mean()),
                      "converged": bool(info["converged"].all())}), flush=True)
    return 0


def serve_mode(args):
    """Poisson stream of solve requests through the continuous-batching server."""
    from paper_2111_01730_amd import serving
    from paper_2111_01730_amd.hodbf import P_FP32
    from synth.workloads import request_inputs, serving_requests
    box = {16: 1.0, 32: 4.0, 64: 8.0}
    sizes = [((n, n, n), box[n]) for n in (int(v) for v in args.serve_sizes.split(","))]
    stream = serving_requests(seed=4, count=args.serve_requests, rate=args.serve_rate, sizes=sizes)
    reqs = []
    for r in stream:
        inp = request_inputs(r)
        reqs.append(serving.Request(id=r["id"], grid=inp["grid"], dirs=inp["dirs"],
                                    arrival=r["arrival"], tol=TOL_SOL))
    srv = serving.Server(hbm_budget=200 << 30, slots=args.serve_slots, max_rhs=64,
                         tol_con=1e-4, tol_fact=args.tol_fact, precond=P_FP32, build_slots=3)
    # operators of the scatterer pool are built first (resident), then the stream plays
    tb = time.perf_counter()
    seen = {}
    for q in reqs:
        seen.setdefault(serving.scatterer_key(q.grid), q.grid)
    build_times = srv.preload(list(seen.values()))
    build_wall = time.perf_counter() - tb
    log(f"[serve] {len(seen)} operators resident after {build_wall:.1f} s")
    t0 = time.perf_counter()
    res = serving.replay(srv, reqs)
    wall = time.perf_counter() - t0
    log_ = list(srv.log)
    srv.close()
    summ = serving.summarize(res, wall)
    out = {"mode": "serve", "workload": f"{args.serve_requests} requests, sizes {args.serve_sizes}, "
                                        f"3 scatterers per size, eps_r U[1,12], 1-16 RHS, "
                                        f"Poisson rate {args.serve_rate}/s",
           **summ, "batches": len(log_), "operators": len(seen),
           "operator_build_s": build_times, "operators_resident_after_s": build_wall,
           "slots": args.serve_slots, "tol_fact": args.tol_fact}
    print(json.dumps(out), flush=True)
    return 0


def config_mode(args):
    """One named workload end to end: build, forward and preconditioner applies, and a
    batched FP32-preconditioned solve (iterations, time, true residual)."""
    import torch

    from paper_2111_01730_amd.hodbf import P_FP32, Operator
    from synth import config
    cfg = config(args.config)
    g = cfg["grid"]
    R = cfg["nrhs"]
    tol = cfg["tol"]
    t0 = time.perf_counter()
    op = Operator(g, tol_con=tol, tol_fact=args.tol_fact, precond=P_FP32,
                  precond_min_level=args.precond_min_level, seed=cfg["seed"])
    build_s = time.perf_counter() - t0
    st = op.stats()
    log(f"[build] {build_s:.1f}s {st}")
    b = op.plane_wave(cfg["dirs"])
    perm = torch.as_tensor(op.perm().astype(np.int64), device="cuda")
    xt = b[perm].to(torch.complex64).contiguous()
    times = {}
    for name, which in (("forward", 0), ("precond_fp32", 2), ("precond_fp32_split", 6)):
        for _ in range(2):
            op.apply_tree(xt, which)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(5):
            op.apply_tree(xt, which)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - ta) / 5
    # the all-FP32 solve and the mixed one (FP32 forward, split-BF16 preconditioner)
    solves = {}
    for arith in ("fp32", "fp32_split"):
        torch.cuda.synchronize()
        tsol = time.perf_counter()
        x, info = op.solve(b, tol=tol, restart=args.restart, max_iter=args.max_iter,
                           use_precond=arith)
        torch.cuda.synchronize()
        dt = time.perf_counter() - tsol
        solves[arith] = {"solve_s": dt, "solves_per_s": R / dt,
                         "iters_max": int(info["iters"].max()),
                         "iters_mean": float(info["iters"].mean()),
                         "converged": bool(info["converged"].all()),
                         "relres_max": float(info["relres"].max())}
        log(f"[solve {arith}] {solves[arith]}")
    solve_s = solves["fp32"]["solve_s"]
    out = {"mode": "config", "config": args.config, "n": g.n, "nrhs": R, "tol_con": tol,
           "tol_fact": args.tol_fact, "precond_min_level": args.precond_min_level,
           "build_s": build_s, "forward_build_s": st["build_seconds"],
           "precond_build_s": st["precond_seconds"], "entries_fwd": st["entries_fwd"],
           "entries_pre": st["entries_pre"], "max_rank": st["max_rank"],
           "bytes_total": st["bytes_total"],
           "forward_apply_ms": times["forward"] * 1e3,
           "forward_gflops": 8.0 * R * st["entries_fwd"] / times["forward"] / 1e9,
           "precond_apply_ms": times["precond_fp32"] * 1e3,
           "precond_apply_ms_split": times["precond_fp32_split"] * 1e3,
           "solve_s": solve_s, "solves": solves, "restart": args.restart}
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol-fact", type=float, default=1e-5)
    ap.add_argument("--mode", choices=["solve", "solves", "apply", "serve", "config", "oracle"],
                    default="solve")
    ap.add_argument("--config", default="c3_sphere_64", help="workload of --mode config")
    ap.add_argument("--precond-min-level", type=int, default=0)
    ap.add_argument("--precond-dense-levels", type=int, default=4,
                    help="solve / apply modes: tree levels (above the leaves) whose "
                         "preconditioner factors are replaced by dense node inverses")
    ap.add_argument("--restart", type=int, default=20)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--serve-sizes", default="16,32", help="cube sides drawn by requests")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--variant-max-iter", type=int, default=300)
    ap.add_argument("--plain-rhs", type=int, default=4, help="columns timed in the plain form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 64^3 forward apply")
    ap.add_argument("--cpu-baseline-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--apply-nrhs", type=int, default=0,
                    help="--mode apply: right-hand sides (0: the workload's 64)")
    ap.add_argument("--user-order", action="store_true",
                    help="--mode apply, which 0: hodbf_apply on the user's complex FP64 "
                         "vectors (gather, apply, scatter) instead of the tree-order apply")
    ap.add_argument("--which", type=int, default=0,
                    help="--mode apply: 0 forward, 6 preconditioner on split-BF16 arithmetic")
    args = ap.parse_args()

    if args.cpu_baseline_leg:
        print(json.dumps(cpu_baseline_leg(20.0, WORKLOAD)))
        return 0
    if args.mode == "oracle":  # host only, no GPU
        print(json.dumps(oracle_mode(args)))
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "hodbf runs on one GPU (multi-GPU sharding is a design, not built); --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import torch

    from paper_2111_01730_amd.hodbf import P_BF16, P_FP16, P_FP32, P_NONE, Operator
    from synth import config

    torch.cuda.set_device(0)
    cfg = config(WORKLOAD)
    g = cfg["grid"]
    R = cfg["nrhs"]
    if args.mode == "apply":
        return apply_mode(args, cfg, Operator, P_NONE)
    if args.mode == "solves":
        return solves_mode(args, cfg, Operator)
    if args.mode == "serve":
        return serve_mode(args)
    if args.mode == "config":
        # multi-minute constructions: the library's progress messages go to stderr
        os.environ.setdefault("HODBF_LOG", "1")
        return config_mode(args)
    t0 = time.perf_counter()
    op = Operator(g, tol_con=cfg["tol"], tol_fact=args.tol_fact, precond=P_FP32 | P_BF16 | P_FP16,
                  seed=cfg["seed"],
                  precond_dense_levels=args.precond_dense_levels)
    build_s = time.perf_counter() - t0
    st = op.stats()
    log(f"[build] {build_s:.1f}s stats={st}")
    b = op.plane_wave(cfg["dirs"])
    perm = torch.as_tensor(op.perm().astype(np.int64), device="cuda")
    xt = b[perm].to(torch.complex64).contiguous()  # tree order, RHS interleaved
    stream = torch.cuda.current_stream()

    def time_apply(which, reps):
        for _ in range(2):
            op.apply_tree(xt, which)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            op.apply_tree(xt, which)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    # the mixed form: FP32 forward on FP32 MFMA, the preconditioner's FP32 copy on
    # split-BF16 MFMA with FP32 accumulation, FP64 Krylov; R columns batched
    MIXED = "fp32_split"
    t_fwd = time_apply(0, args.apply_reps)
    t_pre = {c: time_apply(w, args.apply_reps)
             for c, w in ((MIXED, 6), ("fp32", 2), ("fp16", 4), ("bf16", 3))}
    flops_fwd = 8.0 * R * st["entries_fwd"]
    log(f"[apply] fwd {t_fwd * 1e3:.3f} ms ({flops_fwd / t_fwd / 1e9:.1f} GFLOP/s), precond "
        + ", ".join(f"{c} {t * 1e3:.3f} ms" for c, t in t_pre.items()))

    # warmup solves
    for _ in range(args.warmup):
        _, info = op.solve(b, tol=TOL_SOL, use_precond=MIXED)
    torch.cuda.synchronize()
    iters = []
    conv = True
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        x, info = op.solve(b, tol=TOL_SOL, use_precond=MIXED)
        iters.append(int(info["iters"].max()))
        conv = conv and bool(info["converged"].all())
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - ts) / args.steps
    solves_per_s = R / t_step
    iters_mean = float(info["iters"].mean())
    log(f"[solve batched {MIXED}] {t_step * 1e3:.1f} ms/step, iters max {iters}, "
        f"mean {iters_mean:.1f}, converged {conv}, relres max {info['relres'].max():.2e}")

    # the other preconditioner arithmetics on the same batch (bounded)
    variants = {}
    for c in ("fp32", "fp16", "bf16"):
        torch.cuda.synchronize()
        tv = time.perf_counter()
        _, vi = op.solve(b, tol=TOL_SOL, use_precond=c, max_iter=args.variant_max_iter)
        torch.cuda.synchronize()
        dt = time.perf_counter() - tv
        variants[c] = {"converged": bool(vi["converged"].all()), "iters_max": int(vi["iters"].max()),
                       "iters_mean": float(vi["iters"].mean()), "relres_max": float(vi["relres"].max()),
                       "seconds": dt, "solves_per_s": (R / dt) if vi["converged"].all() else 0.0,
                       "precond_apply_ms": t_pre[c] * 1e3}
        log(f"[solve batched {c}] {variants[c]}")

    # plain form: FP32 preconditioner, one column at a time, every product with Z in FP32
    npl = min(args.plain_rhs, R)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plain_iters = []
    for q in range(npl):
        _, pinfo = op.solve(b[:, q].contiguous(), tol=TOL_SOL, use_precond="fp32",
                            fp32_only=True)
        plain_iters.append(int(pinfo["iters"][0]))
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - tp) / npl
    plain_solves_per_s = 1.0 / t_plain
    log(f"[solve plain] {t_plain * 1e3:.1f} ms/column, iters {plain_iters}")

    cpu = cpu_1core = None
    if not args.no_cpu_baseline:
        legs = {}
        for tag in ("all", "1"):
            env = dict(os.environ)
            if tag == "1":
                env.update(OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-leg"],
                               capture_output=True, text=True, env=env, timeout=600)
            legs[tag] = json.loads(r.stdout.strip().splitlines()[-1])
            log(f"[cpu oracle, threads {tag}] {legs[tag]}")

        def baseline(leg, allowed):
            steps = leg["projected_steps"]
            how = ("converged" if leg["converged"] else
                   f"projected from the log-linear trend of its residual history, "
                   f"{leg['residual']:.2e} after {leg['steps_run']} steps")
            return {"value": leg["solves_per_s"], "unit": "solves/s",
                    "cores": max(1, int(round(leg["threads_busy"]))), "kind": "oracle",
                    "threads_allowed": allowed, "host_cpus": leg["host_cpus"],
                    "sample": (f"{leg['steps_run']} FGMRES(20) steps of the oracle (its FFT-exact "
                               f"FP64 product, modified Gram-Schmidt, no preconditioner: its "
                               f"multiplicative inverse is a dense construction out of reach at "
                               f"this size) on plane wave 0 of this workload in "
                               f"{leg['seconds']:.1f} s ({leg['sec_per_step'] * 1e3:.1f} ms per "
                               f"step, {leg['cpu_seconds']:.1f} s of CPU time); steps to 1e-4: "
                               f"{steps:.0f}, {how}; solves/s = 1 / (s per step x steps)")}

        cpu = baseline(legs["all"], "all")
        cpu_1core = baseline(legs["1"], 1)

    # roofline of a grouped kernel over one apply at R columns: algorithmic flops 8 R E and
    # bytes 8 E (factors) + 8 R io_rows (per launch: output rows once, distinct input rows
    # once); the bound is the side of the ridge the arithmetic intensity falls on
    same_src = sources_sha256() == MEASURED_TRAFFIC["sources_sha256"]

    def roofline(entries, io_rows, launches, t, peak_tflops, kernel, key):
        fl = 8.0 * R * entries
        by = 8.0 * entries + 8.0 * R * io_rows
        ai = fl / by
        ridge = peak_tflops * 1e12 / (PEAK_HBM_GBS * 1e9)
        mt = MEASURED_TRAFFIC[key]
        traffic = (mt["bytes_per_apply"] / mt["launches_per_apply"]
                   if same_src and mt["bytes_per_apply"] else None)
        if ai < ridge:
            ach = by / t / 1e9
            r = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": ach / PEAK_HBM_GBS}
        else:
            ach = fl / t / 1e12
            r = {"bound": "mfma", "achieved": ach, "peak": peak_tflops, "unit": "TFLOP/s",
                 "frac": ach / peak_tflops}
        r.update({"traffic": traffic, "traffic_unit": "bytes per launch",
                  "algorithmic_bytes_per_launch": by / launches,
                  "algorithmic_flops_per_launch": fl / launches,
                  "arithmetic_intensity": ai, "ridge": ridge, "tflops": fl / t / 1e12,
                  "gbs": by / t / 1e9, "kernel": kernel, "launches_per_apply": launches,
                  "avg_launch_us": t / launches * 1e6})
        return r

    # the dominant kernel of the timed solves is the preconditioner's (about two thirds
    # of a step); the forward kernel's roofline is reported beside it
    roof = roofline(st["entries_pre"], st["io_rows_pre"], st["pre_stages"], t_pre[MIXED],
                    PEAK_BF16_MFMA_TFLOPS,
                    "k_grouped_mfma_s3 (preconditioner apply, FP32 factors on split-BF16 MFMA, "
                    "all launches)", "precond_s3")
    roof["block_sums"] = precond_block_sums(op, R)
    copy_gbs = measured_copy_gbs()
    roof["measured_peaks"] = {"hbm_copy_gbs": copy_gbs}
    roof_fwd = roofline(st["entries_fwd"], st["io_rows_fwd"], st["fwd_stages"], t_fwd,
                        PEAK_FP32_MFMA_TFLOPS, "k_grouped_mfma_f32 (forward apply, all launches)",
                        "forward_f32")
    roof_fwd["per_stage"] = stage_roofline(op, st, R, t_fwd)
    roof_fwd["mfma_frac"] = flops_fwd / t_fwd / 1e12 / PEAK_FP32_MFMA_TFLOPS
    # the 64^3 sphere's forward apply (its preconditioner is beyond these minutes): the
    # apply GFLOP/s half of the metric on the larger configuration
    c3 = None
    if not args.no_c3:
        del op
        torch.cuda.empty_cache()
        c3 = c3_forward(Operator, P_NONE, args.apply_reps)
        log(f"[c3 forward] {c3}")
    out = {
        "metric": "HOD-BF apply GFLOP/s + solves/sec at 1e-4 rel. residual, mixed vs plain FP32",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 forward on f32 mfma / c64 precond on split-bf16 mfma, f32 accumulate / c128 krylov",
        "data": "synthetic",
        "config": {"workload": "32^3 voxels, 4-wavelength cube, eps_r iid U[2,10], 64 plane waves",
                   "n": g.n, "nrhs": R, "leaf": 64, "tol_con": cfg["tol"],
                   "tol_fact": args.tol_fact, "tol_sol": TOL_SOL,
                   "precond_dense_levels": args.precond_dense_levels, "parallelism": "1 GPU"},
        "apply_gflops": flops_fwd / t_fwd / 1e9,
        "apply_ms": t_fwd * 1e3,
        "precond_apply_ms": t_pre[MIXED] * 1e3,
        "precond_apply_ms_fp32": t_pre["fp32"] * 1e3,
        "precond_arithmetic": MIXED,
        "batched_solves_per_s": solves_per_s,
        "plain_fp32_solves_per_s": plain_solves_per_s,
        "batched_vs_plain": solves_per_s / plain_solves_per_s,
        "other_precond_arithmetic": variants,
        "iters_batched_max": max(iters),
        "iters_batched_mean": iters_mean,
        "iters_plain": plain_iters,
        "converged": conv,
        "build_s": build_s,
        "precond_build_s": st["precond_seconds"],
        "entries_fwd": st["entries_fwd"],
        "entries_pre": st["entries_pre"],
        "max_rank": st["max_rank"],
        "roofline": roof,
        "roofline_forward": roof_fwd,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu_1core,
        "c3_sphere_64_forward": c3,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
