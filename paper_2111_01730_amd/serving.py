"""Continuous-batching solve service on one GPU.

Requests (a scatterer: grid + permittivity, and a set of plane-wave directions) arrive
over time.  The scheduler

* keeps compressed operators resident in HBM, keyed by the scatterer, and evicts idle
  ones least-recently-used when the device-memory budget needs room;
* builds missing operators on a separate builder pool (so construction never holds a
  solve slot), in arrival order, when their estimated size fits the budget;
* admits pending requests whose operator is resident, in arrival order, whenever a
  solve slot is free and their solve workspace fits the budget;
* merges every pending request that targets the same resident operator into one
  batched FGMRES solve (their right-hand sides stacked, up to ``max_rhs`` columns);
* runs each batch on a worker thread with its own HIP stream, so batches of different
  operators overlap on the device.

A request's result does not depend on what it was batched with beyond floating-point
summation order: every right-hand side is an independent column of the FGMRES solve
(per-column Gram-Schmidt, rotations and stopping test).

All compute is in ``libhodbf.so``; this module only schedules calls.
"""
from __future__ import annotations

import dataclasses
import hashlib
import threading
import time
from collections import OrderedDict
from concurrent.futures import Future, ThreadPoolExecutor

import numpy as np
import torch

from .hodbf import P_FP32, Operator


@dataclasses.dataclass
class Request:
    id: int
    grid: object          # synth.workloads.Grid-like: nx, ny, nz, h, k0, eps
    dirs: np.ndarray      # (R, 3) unit propagation directions
    arrival: float = 0.0  # seconds after the start of a replayed stream
    tol: float = 1e-4


@dataclasses.dataclass
class Result:
    id: int
    x: np.ndarray         # (N, R) complex128 solution in the user's voxel order
    iters: np.ndarray
    relres: np.ndarray
    converged: bool
    submitted: float
    started: float
    finished: float
    batch_size: int       # requests sharing the solve
    batch_rhs: int        # right-hand sides in that solve
    built: bool           # reserved (construction runs on the builder pool)

    @property
    def latency(self) -> float:
        return self.finished - self.submitted


def scatterer_key(grid) -> str:
    h = hashlib.sha1()
    h.update(np.array([grid.nx, grid.ny, grid.nz], dtype=np.int64).tobytes())
    h.update(np.array([grid.h, grid.k0], dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(grid.eps, dtype=np.complex128).tobytes())
    return h.hexdigest()


def solve_workspace_bytes(n: int, nrhs: int, restart: int) -> int:
    """Estimate of one batch's device memory before its operator exists: the solve's
    workspace (Krylov basis (restart + 1) x 16, preconditioned basis restart x 8, six
    vectors, column staging, an apply workspace taken as 4 N rows) plus the right-hand
    sides and solutions, bytes per unknown and column, and 64 MiB for the rest.  Once the
    operator is built, ``batch_bytes`` asks the library for the exact figure."""
    per = (restart + 1) * 16 + restart * 8 + 6 * 16 + 16 + 4 * 8 + 2 * 16
    return int(n) * int(nrhs) * per + (64 << 20)


def batch_bytes(op, nrhs: int, restart: int, use_precond) -> int:
    """Device memory of one batched solve on a built operator: the library's solve
    workspace for these arguments plus the right-hand sides and the solutions (complex
    FP64, N x nrhs each)."""
    return int(op.solve_workspace(nrhs, restart, use_precond)) + 2 * 16 * int(op.n) * int(nrhs)


class Server:
    def __init__(self, hbm_budget: int, slots: int = 4, max_rhs: int = 64, tol_con: float = 1e-4,
                 tol_fact: float = 1e-4, precond: int = P_FP32, restart: int = 20,
                 max_iter: int = 3000, est_bytes_per_unknown: float = 90_000.0,
                 operator_factory=None, build_slots: int = 1, use_precond="fp32_split"):
        self.budget = int(hbm_budget)
        self.slots = slots
        self.max_rhs = max_rhs
        self.build_kw = dict(tol_con=tol_con, tol_fact=tol_fact, precond=precond)
        self.restart = restart
        self.max_iter = max_iter
        # preconditioner arithmetic of every solve (Operator.solve's use_precond); the
        # default is the mixed form: the FP32 copy on split-BF16 MFMA
        self.use_precond = use_precond
        self.est_per_unknown = est_bytes_per_unknown  # until a real build reports its size
        self._lock = threading.Condition()
        self._pending: list = []              # (request, future, submitted)
        self._ops: "OrderedDict[str, dict]" = OrderedDict()  # key -> {op, bytes, busy}
        self._reserved = 0                   # bytes promised to running batches
        self._running = 0
        self._closed = False
        self._factory = operator_factory or Operator
        self.build_slots = build_slots
        self._building = 0
        self.builds = 0
        self._builder = ThreadPoolExecutor(max_workers=build_slots)
        self._pool = ThreadPoolExecutor(max_workers=slots)
        # one HIP stream per worker slot (default priority); None without a GPU
        self._streams = [torch.cuda.Stream() if torch.cuda.is_available() else None
                         for _ in range(slots)]
        self._free_streams = list(range(slots))
        self._sched = threading.Thread(target=self._loop, daemon=True)
        self.log: list = []
        self._sched.start()

    # ------------------------------------------------------------------ public
    def submit(self, req: Request) -> Future:
        fut: Future = Future()
        if not 1 <= len(req.dirs) <= self.max_rhs:
            # a request wider than one batch could never be admitted
            fut.set_exception(ValueError(
                f"request {req.id}: {len(req.dirs)} right-hand sides, 1..{self.max_rhs} allowed"))
            return fut
        key = scatterer_key(req.grid)
        with self._lock:
            self._pending.append((req, fut, time.perf_counter(), key))
            self._lock.notify_all()
        return fut

    def close(self):
        with self._lock:
            self._closed = True
            self._lock.notify_all()
        self._sched.join()
        self._builder.shutdown(wait=True)
        self._pool.shutdown(wait=True)
        for ent in self._ops.values():
            if ent["op"] is not None:
                ent["op"].close()
        self._ops.clear()

    def preload(self, grids) -> list:
        """Build the operators of these scatterers into the resident cache now, on the
        builder pool (blocking); returns each build's seconds."""
        futs = []

        def timed(key, grid):
            t0 = time.perf_counter()
            self._build(key, grid)
            return time.perf_counter() - t0

        for grid in grids:
            key = scatterer_key(grid)
            with self._lock:
                if key in self._ops:
                    continue
                self._ops[key] = {"op": None, "bytes": self._estimate_op_bytes(grid), "busy": 0}
                self._building += 1
            futs.append(self._builder.submit(timed, key, grid))
        return [f.result() for f in futs]

    def resident_bytes(self) -> int:
        return sum(e["bytes"] for e in self._ops.values())

    # ------------------------------------------------------------------ scheduler
    def _estimate_op_bytes(self, grid) -> int:
        return int(self.est_per_unknown * grid.n)

    def _try_evict(self, need: int, keep=None) -> bool:
        """Drop idle resident operators, least recently used first, until need fits.
        The operator under ``keep`` (the one a batch is about to use) is never dropped."""
        while self.resident_bytes() + self._reserved + need > self.budget:
            idle = [k for k, e in self._ops.items()
                    if e["op"] is not None and e["busy"] == 0 and k != keep]
            if not idle:
                return False
            self._ops.pop(idle[0])["op"].close()
        return True

    def _fail_pending(self, exc: BaseException):
        for item in list(self._pending):
            self._pending.remove(item)
            if not item[1].done():
                item[1].set_exception(exc)

    def _loop(self):
        with self._lock:
            while True:
                if self._closed and not self._pending and self._running == 0 and self._building == 0:
                    return
                try:
                    acted = self._tick()
                except Exception as e:  # a scheduler bug must not strand the waiting requests
                    self._fail_pending(e)
                    acted = True
                if not acted:
                    self._lock.wait(timeout=0.05)

    def _tick(self) -> bool:
        """One pass of the scheduler under the lock; True if it changed anything."""
        acted = False
        # 1. start builds for pending scatterers that are neither resident nor
        #    being built (own pool: builds never hold a solve slot)
        if self._building < self.build_slots:
            for req0, _, _, key in self._pending:
                if key in self._ops:
                    continue
                need = self._estimate_op_bytes(req0.grid)
                if need + solve_workspace_bytes(req0.grid.n, 1, self.restart) > self.budget:
                    for item in [it for it in self._pending if it[3] == key]:
                        self._pending.remove(item)
                        item[1].set_exception(MemoryError(
                            f"operator needs about {need} bytes, budget {self.budget}"))
                    acted = True
                    break
                if self._try_evict(need):
                    self._ops[key] = {"op": None, "bytes": need, "busy": 0}
                    self._building += 1
                    self._builder.submit(self._build, key, req0.grid)
                    acted = True
                break  # oldest first; wait for memory otherwise
        # 2. solve: the oldest request whose operator is resident leads a batch of
        #    every pending request for that scatterer, up to max_rhs columns
        if self._free_streams:
            for req0, _, _, key in self._pending:
                ent = self._ops.get(key)
                if ent is None or ent["op"] is None:
                    continue
                batch, cols = [], 0
                for item in self._pending:
                    if item[3] == key and cols + len(item[0].dirs) <= self.max_rhs:
                        batch.append(item)
                        cols += len(item[0].dirs)
                try:
                    ws = batch_bytes(ent["op"], cols, self.restart, self.use_precond)
                except Exception as e:  # e.g. a preconditioner copy the operator lacks
                    for item in batch:
                        self._pending.remove(item)
                        item[1].set_exception(e)
                    acted = True
                    break
                if ws > self.budget:
                    for item in batch:
                        self._pending.remove(item)
                        item[1].set_exception(MemoryError(
                            f"solve needs {ws} bytes, budget {self.budget}"))
                    acted = True
                elif self._try_evict(ws, keep=key):
                    for item in batch:
                        self._pending.remove(item)
                    self._reserved += ws
                    self._running += 1
                    ent["busy"] += 1
                    self._ops.move_to_end(key)
                    sidx = self._free_streams.pop()
                    self._pool.submit(self._run_batch, key, batch, ws, sidx)
                    acted = True
                break
        return acted

    # ------------------------------------------------------------------ workers
    def _build(self, key, grid):
        try:
            stream = torch.cuda.Stream() if torch.cuda.is_available() else None
            ctx = torch.cuda.stream(stream) if stream is not None else _nullctx()
            with ctx:
                op = self._factory(grid, **self.build_kw)
            if stream is not None:
                stream.synchronize()
            nbytes = op.stats()["bytes_total"]
            with self._lock:
                self._ops[key]["op"] = op
                self._ops[key]["bytes"] = nbytes
                self.builds += 1
                # learn the real size for the estimates of later builds
                self.est_per_unknown = nbytes / grid.n * 1.1
        except Exception as e:
            with self._lock:
                self._ops.pop(key, None)
                for item in [it for it in self._pending if it[3] == key]:
                    self._pending.remove(item)
                    item[1].set_exception(e)
        finally:
            with self._lock:
                self._building -= 1
                self._lock.notify_all()

    def _run_batch(self, key, batch, ws, sidx):
        stream = self._streams[sidx]
        t_start = time.perf_counter()
        try:
            ctx = torch.cuda.stream(stream) if stream is not None else _nullctx()
            with ctx:
                with self._lock:
                    op = self._ops[key]["op"]
                dirs = np.concatenate([item[0].dirs for item in batch], axis=0)
                b = op.plane_wave(dirs)
                tol = min(item[0].tol for item in batch)
                x, info = op.solve(b, tol=tol, restart=self.restart, max_iter=self.max_iter,
                                   use_precond=self.use_precond)
                xh = x.cpu().numpy()
            if stream is not None:
                stream.synchronize()
            t_end = time.perf_counter()
            c = 0
            for req, fut, submitted, _ in batch:
                r = len(req.dirs)
                sl = slice(c, c + r)
                c += r
                fut.set_result(Result(req.id, xh[:, sl], info["iters"][sl], info["relres"][sl],
                                      bool(info["converged"][sl].all()), submitted, t_start,
                                      t_end, len(batch), len(dirs), False))
            self.log.append(dict(key=key[:8], requests=len(batch), rhs=len(dirs),
                                 start=t_start, end=t_end))
        except Exception as e:  # surface the failure on every request of the batch
            for _, fut, _, _ in batch:
                if not fut.done():
                    fut.set_exception(e)
        finally:
            with self._lock:
                if key in self._ops:
                    self._ops[key]["busy"] -= 1
                self._reserved -= ws
                self._running -= 1
                self._free_streams.append(sidx)
                self._lock.notify_all()


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def replay(server: Server, requests: list, time_scale: float = 1.0) -> list:
    """Submit requests at their arrival times (scaled) and wait for every result."""
    t0 = time.perf_counter()
    futs = []
    for req in sorted(requests, key=lambda r: r.arrival):
        delay = req.arrival * time_scale - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(req))
    return [f.result() for f in futs]


def summarize(results: list, wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    rhs = sum(len(r.iters) for r in results)
    return dict(requests=len(results), rhs=rhs, wall_s=wall,
                solves_per_s=rhs / wall if wall > 0 else 0.0,
                p50_latency_s=float(np.percentile(lat, 50)),
                p99_latency_s=float(np.percentile(lat, 99)),
                all_converged=all(r.converged for r in results),
                mean_batch_requests=float(np.mean([r.batch_size for r in results])))
