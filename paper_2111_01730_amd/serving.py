"""Continuous-batching solve service on one GPU.

Requests (a scatterer: grid + permittivity, and a set of plane-wave directions) arrive
over time.  The scheduler

* keeps compressed operators resident in HBM, keyed by the scatterer, and evicts idle
  ones least-recently-used when the device-memory budget needs room;
* admits pending requests in arrival order whenever a worker slot is free and the
  memory they need (operator, if not resident, plus solve workspace) fits the budget;
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
    built: bool           # this request's batch had to build the operator

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
    """Device scratch of one vie_solve (Krylov basis, preconditioned basis, vectors)."""
    per = (restart + 1) * 16 + restart * 8 + 4 * 16 + 2 * 8
    return int(n) * int(nrhs) * per + (64 << 20)


class Server:
    def __init__(self, hbm_budget: int, slots: int = 4, max_rhs: int = 64, tol_con: float = 1e-4,
                 tol_fact: float = 1e-4, precond: int = P_FP32, restart: int = 20,
                 max_iter: int = 3000, est_bytes_per_unknown: float = 90_000.0,
                 operator_factory=None):
        self.budget = int(hbm_budget)
        self.slots = slots
        self.max_rhs = max_rhs
        self.build_kw = dict(tol_con=tol_con, tol_fact=tol_fact, precond=precond)
        self.restart = restart
        self.max_iter = max_iter
        self.est_per_unknown = est_bytes_per_unknown  # until a real build reports its size
        self._lock = threading.Condition()
        self._pending: list = []              # (request, future, submitted)
        self._ops: "OrderedDict[str, dict]" = OrderedDict()  # key -> {op, bytes, busy}
        self._reserved = 0                   # bytes promised to running batches
        self._running = 0
        self._closed = False
        self._factory = operator_factory or Operator
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
        self._pool.shutdown(wait=True)
        for ent in self._ops.values():
            if ent["op"] is not None:
                ent["op"].close()
        self._ops.clear()

    def resident_bytes(self) -> int:
        return sum(e["bytes"] for e in self._ops.values())

    # ------------------------------------------------------------------ scheduler
    def _estimate_op_bytes(self, grid) -> int:
        return int(self.est_per_unknown * grid.n)

    def _try_evict(self, need: int) -> bool:
        """Drop idle resident operators, least recently used first, until need fits."""
        while self.resident_bytes() + self._reserved + need > self.budget:
            idle = [k for k, e in self._ops.items() if e["op"] is not None and e["busy"] == 0]
            if not idle:
                return False
            self._ops.pop(idle[0])["op"].close()
        return True

    def _loop(self):
        with self._lock:
            while True:
                if self._closed and not self._pending and self._running == 0:
                    return
                launched = False
                if self._free_streams and self._pending:
                    for req0, _, _, key in self._pending:
                        ent = self._ops.get(key)
                        if ent is not None and ent["op"] is None:
                            continue  # its operator is being built: join a later batch
                        # the oldest eligible request leads; its batch takes every pending
                        # request for the same scatterer, in arrival order, up to max_rhs
                        batch, cols = [], 0
                        for item in self._pending:
                            r = item[0]
                            if item[3] == key and cols + len(r.dirs) <= self.max_rhs:
                                batch.append(item)
                                cols += len(r.dirs)
                        ws = solve_workspace_bytes(req0.grid.n, cols, self.restart)
                        op_need = 0 if ent is not None else self._estimate_op_bytes(req0.grid)
                        if ws + op_need > self.budget:
                            for item in batch:  # can never fit: fail these requests
                                self._pending.remove(item)
                                item[1].set_exception(MemoryError(
                                    f"request needs {ws + op_need} bytes, budget {self.budget}"))
                            launched = True
                        elif self._try_evict(ws + op_need):
                            for item in batch:
                                self._pending.remove(item)
                            self._reserved += ws
                            self._running += 1
                            if ent is not None:
                                ent["busy"] += 1
                                self._ops.move_to_end(key)
                            else:  # placeholder until the worker has built it
                                self._ops[key] = {"op": None, "bytes": op_need, "busy": 1}
                            sidx = self._free_streams.pop()
                            self._pool.submit(self._run_batch, key, batch, ws, sidx)
                            launched = True
                        break  # first come, first served: only the oldest eligible request
                if not launched:
                    self._lock.wait(timeout=0.05)

    # ------------------------------------------------------------------ worker
    def _run_batch(self, key, batch, ws, sidx):
        stream = self._streams[sidx]
        t_start = time.perf_counter()
        built = False
        try:
            req0 = batch[0][0]
            ctx = torch.cuda.stream(stream) if stream is not None else _nullctx()
            with ctx:
                with self._lock:
                    op = self._ops[key]["op"]
                if op is None:
                    op = self._factory(req0.grid, **self.build_kw)
                    nbytes = op.stats()["bytes_total"]
                    built = True
                    with self._lock:
                        self._ops[key]["op"] = op
                        self._ops[key]["bytes"] = nbytes
                        # learn the real size for the estimates of later builds
                        self.est_per_unknown = nbytes / req0.grid.n * 1.1
                dirs = np.concatenate([item[0].dirs for item in batch], axis=0)
                b = op.plane_wave(dirs)
                tol = min(item[0].tol for item in batch)
                x, info = op.solve(b, tol=tol, restart=self.restart, max_iter=self.max_iter,
                                   use_precond=1)
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
                                      t_end, len(batch), len(dirs), built))
            self.log.append(dict(key=key[:8], requests=len(batch), rhs=len(dirs), built=built,
                                 start=t_start, end=t_end))
        except Exception as e:  # surface the failure on every request of the batch
            with self._lock:
                if key in self._ops and self._ops[key]["op"] is None:
                    self._ops.pop(key)
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
