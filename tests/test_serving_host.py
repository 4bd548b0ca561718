"""Scheduler logic of the serving loop on the CPU with a stand-in operator (no GPU):
admission by memory budget, LRU eviction of idle operators, batching of pending
requests that share a scatterer, failure of requests that can never fit."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
serving = pytest.importorskip("paper_2111_01730_amd.serving")
from synth.workloads import make_grid  # noqa: E402


class FakeOp:
    """Stand-in operator: fixed size, solve returns b after a short sleep."""
    builds = 0
    closes = 0
    lock = threading.Lock()

    def __init__(self, grid, **kw):
        with FakeOp.lock:
            FakeOp.builds += 1
        self.n = grid.n
        time.sleep(0.05)

    def stats(self):
        return {"bytes_total": self.n * 1000}

    def solve_workspace(self, nrhs, restart, use_precond):
        return serving.solve_workspace_bytes(self.n, nrhs, restart) - 2 * 16 * self.n * nrhs

    def plane_wave(self, dirs):
        return torch.ones((self.n, len(dirs)), dtype=torch.complex128)

    def solve(self, b, **kw):
        time.sleep(0.05)
        R = b.shape[1]
        return b.clone(), dict(iters=np.ones(R, np.int32), relres=np.zeros(R),
                               converged=np.ones(R, bool), status="OK")

    def close(self):
        with FakeOp.lock:
            FakeOp.closes += 1


def _grid(seed, side=4):
    rng = np.random.default_rng(seed)
    return make_grid(side, side, side, 0.1, rng.uniform(1, 12, side**3))


def _req(i, g, r=2):
    return serving.Request(id=i, grid=g, dirs=np.tile([[0.0, 0.0, -1.0]], (r, 1)))


@pytest.fixture(autouse=True)
def reset():
    FakeOp.builds = FakeOp.closes = 0


def test_batching_and_results():
    g1, g2 = _grid(1), _grid(2)
    n = g1.n
    ws = serving.solve_workspace_bytes(n, 16, 20)
    srv = serving.Server(hbm_budget=10 * (ws + n * 1000), slots=1, operator_factory=FakeOp,
                         est_bytes_per_unknown=1000)
    futs = [srv.submit(_req(0, g1))]  # occupies the single slot (build + solve)
    time.sleep(0.01)
    futs += [srv.submit(_req(i, g2 if i % 2 else g1)) for i in range(1, 7)]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    assert [r.id for r in res] == list(range(7))
    assert all(r.converged and r.x.shape == (n, 2) for r in res)
    # pending requests for one scatterer were merged into one solve (request 0 waits
    # for its operator's build, so it joins the later requests for the same scatterer)
    assert max(r.batch_size for r in res) >= 3
    assert sum(1 for b in srv.log) <= 4
    assert FakeOp.builds == 2  # each scatterer built once, then resident


def test_budget_evicts_idle_operators():
    gs = [_grid(s) for s in range(3)]
    n = gs[0].n
    ws = serving.solve_workspace_bytes(n, 2, 20)
    # room for one operator and one solve workspace only
    srv = serving.Server(hbm_budget=ws + int(1.5 * n * 1000), slots=2, operator_factory=FakeOp,
                         est_bytes_per_unknown=1000)
    res = [srv.submit(_req(i, gs[i % 3])).result(timeout=10) for i in range(5)]
    srv.close()
    assert all(r.converged for r in res)
    assert FakeOp.builds == 5 and FakeOp.closes == 5  # every switch evicted the previous one
    assert srv.resident_bytes() == 0


def test_request_that_cannot_fit_fails():
    g = _grid(3)
    srv = serving.Server(hbm_budget=1000, slots=1, operator_factory=FakeOp)
    with pytest.raises(MemoryError):
        srv.submit(_req(0, g)).result(timeout=10)
    srv.close()


class NoWorkspaceOp(FakeOp):
    """Stand-in whose library call for the solve's workspace fails (as for a
    preconditioner copy the operator lacks)."""

    def solve_workspace(self, nrhs, restart, use_precond):
        raise RuntimeError("no such preconditioner copy")


def test_failing_workspace_query_fails_the_batch_not_the_scheduler():
    g = _grid(4)
    srv = serving.Server(hbm_budget=1 << 40, slots=1, operator_factory=NoWorkspaceOp,
                         est_bytes_per_unknown=1000)
    with pytest.raises(RuntimeError):
        srv.submit(_req(0, g)).result(timeout=10)
    # the scheduler is still alive and serves the next request the same way
    with pytest.raises(RuntimeError):
        srv.submit(_req(1, g)).result(timeout=10)
    srv.close()


def test_request_wider_than_a_batch_is_refused():
    g = _grid(5)
    srv = serving.Server(hbm_budget=1 << 40, slots=1, max_rhs=4, operator_factory=FakeOp)
    with pytest.raises(ValueError):
        srv.submit(_req(0, g, r=5)).result(timeout=10)
    assert srv.submit(_req(1, g, r=4)).result(timeout=10).converged
    srv.close()


def test_summary_percentiles():
    res = [serving.Result(i, np.zeros((1, 1)), np.ones(1), np.zeros(1), True, 0.0, 0.0, float(i + 1),
                          1, 1, False) for i in range(100)]
    s = serving.summarize(res, 10.0)
    assert s["rhs"] == 100 and s["solves_per_s"] == 10.0
    assert abs(s["p50_latency_s"] - 50.5) < 1e-9 and s["p99_latency_s"] > 98


def test_eviction_keeps_the_operator_the_batch_will_use():
    """Two resident idle operators fill the budget but for a one-column workspace; a
    two-column request for the least recently used one needs room, which must come from
    evicting the other operator, never the one the batch is about to run on."""
    g1, g2 = _grid(11), _grid(12)
    n = g1.n
    ws1 = serving.solve_workspace_bytes(n, 1, 20)
    srv = serving.Server(hbm_budget=2 * n * 1000 + ws1, slots=1, operator_factory=FakeOp,
                         est_bytes_per_unknown=1000)
    srv.preload([g1, g2])  # g1 is now the least recently used resident operator
    assert FakeOp.builds == 2 and FakeOp.closes == 0
    res = srv.submit(_req(0, g1, r=2)).result(timeout=10)
    assert res.converged and res.x.shape == (n, 2)
    assert FakeOp.closes == 1 and FakeOp.builds == 2  # g2 went; g1 served without a rebuild
    assert srv._sched.is_alive()
    srv.close()


def test_scheduler_error_fails_pending_requests():
    """An exception inside one scheduler pass fails the requests that were waiting
    instead of stranding them (and the scheduler keeps running)."""
    g = _grid(13)
    srv = serving.Server(hbm_budget=1 << 40, slots=1, operator_factory=FakeOp,
                         est_bytes_per_unknown=1000)
    calls = {"n": 0}
    orig = srv._estimate_op_bytes

    def broken(grid):
        calls["n"] += 1
        if calls["n"] == 1:
            raise KeyError("planted scheduler fault")
        return orig(grid)

    srv._estimate_op_bytes = broken
    with pytest.raises(KeyError):
        srv.submit(_req(0, g)).result(timeout=10)
    assert srv.submit(_req(1, g)).result(timeout=10).converged
    srv.close()
