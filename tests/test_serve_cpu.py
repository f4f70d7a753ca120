"""Scheduler logic of the GP-solve server, exercised on the CPU with a test
double in place of the GPU executor (no device work, no second solver
path: the double only sleeps and reports what it was given)."""
import threading
import time

import numpy as np
import pytest

from paper_2605_13209_amd.serve import Executor, RequestTooLarge, Server, SolveRequest, SolveResult


class FakeExecutor(Executor):
    """Footprint = n*n bytes (+ n extra while in flight); run sleeps n/1e5 s."""

    def __init__(self, fail_n=None):
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.active_bytes = 0
        self.max_active_bytes = 0
        self.order = []
        self.cached_runs = []
        self.fail_n = fail_n

    def cache_bytes(self, req):
        return req.n * req.n

    def footprint(self, req, cached):
        return req.n + (0 if cached else req.n * req.n)

    def run(self, req, cached, worker):
        fp = self.footprint(req, cached is not None)
        with self.lock:
            self.active += 1
            self.active_bytes += fp
            self.max_active = max(self.max_active, self.active)
            self.max_active_bytes = max(self.max_active_bytes, self.active_bytes)
            self.order.append(req.rid)
            self.cached_runs.append((req.rid, cached is not None))
        try:
            time.sleep(req.n / 1e5)
            if self.fail_n is not None and req.n == self.fail_n:
                raise ValueError("planted failure")
            return SolveResult(np.zeros((req.n, 1)), 1, True, 0.0, cached is not None, req.t_arrival,
                               time.perf_counter(), time.perf_counter()), {"rid": req.rid}
        finally:
            with self.lock:
                self.active -= 1
                self.active_bytes -= fp


def req(n, rid, key=None):
    return SolveRequest(X=np.zeros((n, 2)), B=np.zeros((n, 1)), key=key, rid=rid)


def test_budget_and_slots_respected():
    ex = FakeExecutor()
    budget = 3 * (1000 * 1000 + 1000)
    with Server(ex, hbm_budget=budget, max_inflight=8, cache=False) as s:
        futs = [s.submit(req(1000, i)) for i in range(12)]
        for f in futs:
            f.result(timeout=30)
    assert ex.max_active_bytes <= budget
    assert ex.max_active == 3


def test_max_inflight_respected():
    ex = FakeExecutor()
    with Server(ex, hbm_budget=1e12, max_inflight=2, cache=False) as s:
        for f in [s.submit(req(500, i)) for i in range(8)]:
            f.result(timeout=30)
    assert ex.max_active == 2


def test_fifo_admission():
    ex = FakeExecutor()
    with Server(ex, hbm_budget=1e12, max_inflight=1, cache=False) as s:
        for f in [s.submit(req(100 + i, i)) for i in range(10)]:
            f.result(timeout=30)
    assert ex.order == list(range(10))


def test_oversized_rejected_immediately():
    ex = FakeExecutor()
    with Server(ex, hbm_budget=10_000, max_inflight=2) as s:
        f = s.submit(req(1000, 0))
        with pytest.raises(RequestTooLarge):
            f.result(timeout=5)
        assert s.stats()["rejected"] == 1
        assert s.submit(req(50, 1)).result(timeout=5).converged


def test_factor_cache_reuse_and_lru_eviction():
    ex = FakeExecutor()
    n = 200
    # room for one cached factor next to one in-flight miss (or two cached)
    budget = 2 * n * n + 4 * n
    with Server(ex, hbm_budget=budget, max_inflight=1, cache=True) as s:
        s.submit(req(n, 0, key="a")).result(timeout=10)
        s.submit(req(n, 1, key="b")).result(timeout=10)
        r = s.submit(req(n, 2, key="a")).result(timeout=10)   # hit
        assert r.reused_factor
        s.submit(req(n, 3, key="c")).result(timeout=10)      # evicts LRU ("b")
        r = s.submit(req(n, 4, key="b")).result(timeout=10)   # miss again
        assert not r.reused_factor
        st = s.stats()
        assert st["evictions"] >= 1 and st["reused_factors"] == 1
        assert s.resident_bytes <= budget
    assert dict(ex.cached_runs)[2] is True and dict(ex.cached_runs)[4] is False


def test_failure_propagates_and_frees_slot():
    ex = FakeExecutor(fail_n=300)
    with Server(ex, hbm_budget=1e12, max_inflight=1, cache=False) as s:
        bad = s.submit(req(300, 0))
        good = s.submit(req(100, 1))
        with pytest.raises(ValueError, match="planted"):
            bad.result(timeout=10)
        assert good.result(timeout=10).converged
        assert s.resident_bytes == 0


def test_stats_latency_fields():
    ex = FakeExecutor()
    with Server(ex, hbm_budget=1e12, max_inflight=4) as s:
        for f in [s.submit(req(300, i)) for i in range(16)]:
            f.result(timeout=30)
        st = s.stats()
    assert st["completed"] == 16
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["req_per_s"] > 0
