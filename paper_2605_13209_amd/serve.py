"""Continuous-batching GP-solve server over the HIP library.

A request is one GP system (features X, hyper-parameters, right-hand sides B)
to be solved to FP64 accuracy.  The server

* admits requests first-in first-out while a slot is free and the request's
  HBM footprint fits the budget next to everything already resident (in-flight
  requests and cached factors; unpinned cached factors are evicted
  least-recently-used first to make room); a request that could never fit is
  rejected at once;
* runs every admitted request on a worker thread with its own HIP stream
  (assemble A, low-precision factorisation, FP64 refinement), so requests
  admitted while others are on the GPU overlap with them on the device;
* keeps factors resident, keyed by the request's matrix key, for repeat
  solves with the same matrix;
* records arrival, admission and completion times for p50/p99 latency.

The kernels are deterministic and a request's schedule depends only on its
own size and precision, so its result is bitwise the same whether it runs
alone or in a mix.

The scheduler (``Server``) only sees the ``Executor`` interface, so its
admission and caching logic can be exercised on the CPU with a test double.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import json
import os
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Hashable, Optional

import numpy as np

__all__ = ["SolveRequest", "SolveResult", "Executor", "HipExecutor", "BatchedHipExecutor", "EngineStepper",
           "Server", "TuningTable", "RequestTooLarge"]


class RequestTooLarge(RuntimeError):
    """The request's footprint exceeds the whole HBM budget."""


@dataclass
class SolveRequest:
    X: np.ndarray                 # n x d features (host, row-major FP64)
    B: np.ndarray                 # n x k right-hand sides (host FP64)
    lengthscale: float = 1.0
    variance: float = 1.0
    noise: float = 0.1
    key: Optional[Hashable] = None  # equal keys promise equal (X, hyper-parameters)
    tol: float = 1e-10
    rid: int = -1
    t_arrival: float = 0.0

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def k(self) -> int:
        return int(self.B.shape[1]) if self.B.ndim == 2 else 1


@dataclass
class SolveResult:
    X: np.ndarray
    iters: int
    converged: bool
    cert: float
    reused_factor: bool
    t_arrival: float
    t_admit: float
    t_done: float
    flops: float = 0.0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class TuningTable:
    """Tile and panel width per (precision, n), from an autotuner table file.

    The file maps precision -> list of [n_max, tile, panel_width] rows sorted
    by n_max; the first row with n <= n_max applies.  Without a file (or
    beyond its last row) the library's defaults are used (tile 0, width 0)."""

    def __init__(self, path: Optional[str] = None):
        self.rows: dict = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.rows = json.load(f).get("table", {})

    def lookup(self, precision: str, n: int) -> tuple[int, int]:
        for n_max, tile, width in self.rows.get(precision, []):
            if n <= n_max:
                return int(tile), int(width)
        return 0, 0


DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x_gfx950.json")


class Executor:
    """What the scheduler needs from a backend."""

    def footprint(self, req: SolveRequest, cached: bool) -> int:
        """Device bytes the request needs while in flight (factor excluded if cached)."""
        raise NotImplementedError

    def cache_bytes(self, req: SolveRequest) -> int:
        """Device bytes a cached factor of this request keeps resident."""
        raise NotImplementedError

    def run(self, req: SolveRequest, cached: Optional[Any], worker: int) -> tuple[SolveResult, Any]:
        """Solve; returns (result, cache entry or None).  ``cached`` is a previous entry."""
        raise NotImplementedError


class HipExecutor(Executor):
    """The GPU backend: gp_assemble -> chol_factor (low precision) -> chol_refine_solve."""

    def __init__(self, precision: str = "fp32", method: str = "ir", device: int = 0, workers: int = 8,
                 table: Optional[TuningTable] = None, max_iter: int = 30):
        import torch
        from . import _native as P
        self.P, self.torch = P, torch
        self.precision, self.method, self.max_iter = precision, method, max_iter
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(workers)]
        self.table = table or TuningTable(DEFAULT_TABLE)

    def _tile(self, n: int) -> tuple[int, int]:
        tile, width = self.table.lookup(self.precision, n)
        return (tile or self.P.chol_tile_default(n, self.precision)), width

    def cache_bytes(self, req: SolveRequest) -> int:
        n = req.n
        tile, _ = self._tile(n)
        return n * n * 8 + n * req.X.shape[1] * 8 + self.P.chol_factor_bytes(n, self.precision, tile)

    def footprint(self, req: SolveRequest, cached: bool) -> int:
        n, k = req.n, req.k
        vec = 3 * n * k * 8 + self.P.chol_refine_bytes(n, k, self.method)
        return vec + (0 if cached else self.cache_bytes(req))

    def run(self, req, cached, worker):
        torch, P = self.torch, self.P
        stream = self.streams[worker % len(self.streams)]
        n = req.n
        t_admit = time.perf_counter()
        with torch.cuda.stream(stream):
            if cached is None:
                Xd = torch.from_numpy(np.ascontiguousarray(req.X, dtype=np.float64)).pin_memory().to(
                    self.device, non_blocking=True)
                A = P.colmajor_empty(n, n, device=self.device)
                P.gp_assemble(Xd, req.lengthscale, req.variance, req.noise, full=False, out=A, stream=stream)
                tile, width = self._tile(n)
                ws = torch.empty(P.chol_factor_bytes(n, self.precision, tile), dtype=torch.uint8,
                                 device=self.device)
                F = P.chol_factor(A, self.precision, tile, workspace=ws, sync=False, stream=stream,
                                  panel_width=width)
                entry = {"A": A, "X": Xd, "ws": ws, "F": F}
                reused = False
            else:
                entry, reused = cached, True
            Bh = np.asfortranarray(req.B.reshape(n, -1), dtype=np.float64)
            Bd = P.to_colmajor(torch.from_numpy(Bh).pin_memory(), device=self.device)
            res = P.chol_refine_solve(entry["F"], Bd, A=entry["A"], noise=req.noise, tol=req.tol,
                                      method=self.method, max_iter=self.max_iter, raise_on_fail=False,
                                      stream=stream)
            Xh = res.X.to("cpu", non_blocking=False).numpy()
        flops = (0 if reused else n ** 3 / 3) + 4.0 * n * n * req.k * (1 + res.iters)
        return (SolveResult(Xh, res.iters, res.converged, res.cert, reused, req.t_arrival, t_admit,
                            time.perf_counter(), flops), entry)


class EngineStepper:
    """Drives a batching engine (step() -> (active, finished), done(job)):
    a thread runs steps while jobs are pending; wait(job) returns once the
    job's last step is enqueued.  An exception in the stepping thread is
    kept and raised in every waiter (and later submitter) instead of leaving
    them waiting; wait() also gives up after `timeout` seconds."""

    def __init__(self, engine, on_thread_start=None, timeout: float = 600.0):
        self.engine = engine
        self.timeout = timeout
        self._cv = threading.Condition()
        self._pending = 0
        self._closing = False
        self._error: Optional[BaseException] = None
        self.steps = 0
        self._on_start = on_thread_start
        self._thread = threading.Thread(target=self._run, name="gp-batch-steps", daemon=True)
        self._thread.start()

    def _run(self):
        try:
            if self._on_start:
                self._on_start()
            while True:
                with self._cv:
                    while self._pending == 0 and not self._closing:
                        self._cv.wait()
                    if self._closing:
                        return
                active, finished = self.engine.step()
                with self._cv:
                    self.steps += 1
                    if finished:
                        self._pending -= finished
                        self._cv.notify_all()
        except BaseException as e:  # noqa: BLE001 - handed to the waiters
            with self._cv:
                self._error = e
                self._cv.notify_all()

    def submit(self, add):
        """Run add() (which registers a job with the engine) and count it."""
        with self._cv:
            if self._error is not None:
                raise RuntimeError("batching engine stopped") from self._error
            job = add()
            self._pending += 1
            self._cv.notify_all()
            return job

    def wait(self, job):
        deadline = time.monotonic() + self.timeout
        with self._cv:
            while not self.engine.done(job):
                if self._error is not None:
                    raise RuntimeError("batching engine stopped") from self._error
                left = deadline - time.monotonic()
                if left <= 0:
                    raise TimeoutError(f"job {job} not finished after {self.timeout} s "
                                       f"({self.steps} steps, {self._pending} pending)")
                self._cv.wait(timeout=min(left, 1.0))

    def close(self):
        """Stop stepping (jobs still pending are left unfinished)."""
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        self._thread.join()


class BatchedHipExecutor(HipExecutor):
    """The GPU backend with continuous batching of the factorisations: every
    admitted request's FP32 factorisation (tile 128) joins the library's
    batching engine (chol_batch_*), whose steps advance all active requests
    by one tile column with one batched diagonal-tile factorisation, panel
    solve and trailing update, captured once in a HIP graph and replayed.
    A stepping thread runs steps while jobs are active; the request's worker
    thread assembles A on its own stream, hands it to the engine, waits for
    its last step and runs the FP64 refinement on its own stream."""

    def __init__(self, method: str = "ir", device: int = 0, workers: int = 8, max_iter: int = 30,
                 max_jobs: int = 64, use_graph: bool = True):
        super().__init__(precision="fp32", method=method, device=device, workers=workers, max_iter=max_iter)
        P = self.P
        self.engine_stream = self.torch.cuda.Stream(device=self.device)
        self.engine = P.BatchEngine(max_jobs=max_jobs, stream=self.engine_stream, use_graph=use_graph,
                                    device=self.device)
        self.stepper = EngineStepper(self.engine, on_thread_start=lambda: self.torch.cuda.set_device(self.device))

    @property
    def steps(self) -> int:
        return self.stepper.steps

    def _tile(self, n: int) -> tuple[int, int]:
        return 128, 1

    def close(self):
        self.stepper.close()
        self.engine.close()

    def run(self, req, cached, worker):
        torch, P = self.torch, self.P
        stream = self.streams[worker % len(self.streams)]
        n = req.n
        t_admit = time.perf_counter()
        with torch.cuda.stream(stream):
            if cached is None:
                Xd = torch.from_numpy(np.ascontiguousarray(req.X, dtype=np.float64)).pin_memory().to(
                    self.device, non_blocking=True)
                A = P.colmajor_empty(n, n, device=self.device)
                P.gp_assemble(Xd, req.lengthscale, req.variance, req.noise, full=False, out=A, stream=stream)
                ws = torch.empty(P.chol_factor_bytes(n, "fp32", 128), dtype=torch.uint8, device=self.device)
                stream.synchronize()  # A ready before the engine's stream packs it
                job = self.stepper.submit(lambda: self.engine.add(A, ws))
                self.stepper.wait(job)
                F = self.engine.take(job)
                entry = {"A": A, "X": Xd, "ws": ws, "F": F}
                reused = False
            else:
                entry, reused = cached, True
            Bh = np.asfortranarray(req.B.reshape(n, -1), dtype=np.float64)
            Bd = P.to_colmajor(torch.from_numpy(Bh).pin_memory(), device=self.device)
            res = P.chol_refine_solve(entry["F"], Bd, A=entry["A"], noise=req.noise, tol=req.tol,
                                      method=self.method, max_iter=self.max_iter, raise_on_fail=False,
                                      stream=stream)
            Xh = res.X.to("cpu", non_blocking=False).numpy()
        flops = (0 if reused else n ** 3 / 3) + 4.0 * n * n * req.k * (1 + res.iters)
        return (SolveResult(Xh, res.iters, res.converged, res.cert, reused, req.t_arrival, t_admit,
                            time.perf_counter(), flops), entry)


@dataclass
class _Cached:
    entry: Any
    nbytes: int
    pins: int = 0


@dataclass
class _Stats:
    results: list = field(default_factory=list)
    rejected: int = 0
    deferred: int = 0         # admissions that had to wait for memory or a slot
    evictions: int = 0


class Server:
    """FIFO admission by HBM footprint and free slots; one worker thread per slot."""

    def __init__(self, executor: Executor, hbm_budget: float = 200e9, max_inflight: int = 8,
                 cache: bool = True):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_inflight = int(max_inflight)
        self.use_cache = cache
        self._lock = threading.Condition()
        self._queue: collections.deque = collections.deque()
        self._inflight = 0
        self._inflight_bytes = 0
        self._cache: "collections.OrderedDict[Hashable, _Cached]" = collections.OrderedDict()
        self._cache_bytes = 0
        self._pool = cf.ThreadPoolExecutor(max_workers=self.max_inflight, thread_name_prefix="gp-solve")
        self._free_workers = list(range(self.max_inflight))
        self._stats = _Stats()
        self._closed = False
        self._sched = threading.Thread(target=self._schedule, name="gp-admit", daemon=True)
        self._sched.start()

    # -- public -------------------------------------------------------------
    def submit(self, req: SolveRequest) -> cf.Future:
        fut: cf.Future = cf.Future()
        req.t_arrival = req.t_arrival or time.perf_counter()
        need = self.ex.footprint(req, cached=False)
        if need > self.budget:
            self._stats.rejected += 1
            fut.set_exception(RequestTooLarge(f"request needs {need} bytes, budget {self.budget}"))
            return fut
        with self._lock:
            if self._closed:
                raise RuntimeError("server closed")
            self._queue.append((req, fut))
            self._lock.notify_all()
        return fut

    def close(self, wait: bool = True):
        with self._lock:
            self._closed = True
            self._lock.notify_all()
        self._sched.join()
        self._pool.shutdown(wait=wait)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def resident_bytes(self) -> int:
        with self._lock:
            return self._inflight_bytes + self._cache_bytes

    def stats(self) -> dict:
        with self._lock:
            res = list(self._stats.results)
            lat = np.array([r.latency for r in res]) * 1e3 if res else np.zeros(0)
            span = (max(r.t_done for r in res) - min(r.t_arrival for r in res)) if res else 0.0
            return {
                "completed": len(res), "rejected": self._stats.rejected, "deferred": self._stats.deferred,
                "evictions": self._stats.evictions, "reused_factors": sum(r.reused_factor for r in res),
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_ms": float(lat.mean()) if len(lat) else None,
                "req_per_s": len(res) / span if span > 0 else None,
                "gflops": sum(r.flops for r in res) / span / 1e9 if span > 0 else None,
                "all_converged": all(r.converged for r in res),
                "max_cert": max((r.cert for r in res), default=None),
            }

    # -- scheduling ---------------------------------------------------------
    def _evict_for(self, need: int) -> bool:
        """Evict unpinned cached factors (LRU first) until `need` more bytes fit."""
        while self._inflight_bytes + self._cache_bytes + need > self.budget:
            victim = next((k for k, c in self._cache.items() if c.pins == 0), None)
            if victim is None:
                return False
            c = self._cache.pop(victim)
            self._cache_bytes -= c.nbytes
            self._stats.evictions += 1
        return True

    def _schedule(self):
        with self._lock:
            while True:
                while not self._closed and not self._admissible():
                    self._lock.wait()
                if self._closed and not self._queue:
                    return
                if not self._queue:
                    continue
                req, fut = self._queue[0]
                if not self._free_workers:
                    self._stats.deferred += 1
                    self._lock.wait()
                    continue
                cached = self._cache.get(req.key) if (self.use_cache and req.key is not None) else None
                need = self.ex.footprint(req, cached=cached is not None)
                if cached is not None:
                    cached.pins += 1  # keep it resident while in use
                if not self._evict_for(need):
                    if cached is not None:
                        cached.pins -= 1
                    self._stats.deferred += 1
                    self._lock.wait()
                    continue
                self._queue.popleft()
                if cached is not None:
                    self._cache.move_to_end(req.key)
                worker = self._free_workers.pop()
                self._inflight += 1
                self._inflight_bytes += need
                self._pool.submit(self._run, req, fut, cached, need, worker)

    def _admissible(self) -> bool:
        return bool(self._queue) and bool(self._free_workers)

    def _run(self, req, fut, cached, need, worker):
        entry = None
        try:
            result, entry = self.ex.run(req, cached.entry if cached is not None else None, worker)
        except BaseException as e:  # noqa: BLE001 - delivered to the caller's future
            with self._lock:
                self._release(req, cached, need, worker, None)
            fut.set_exception(e)
            return
        with self._lock:
            self._stats.results.append(result)
            self._release(req, cached, need, worker, entry)
        fut.set_result(result)

    def _release(self, req, cached, need, worker, entry):
        self._inflight -= 1
        self._inflight_bytes -= need
        self._free_workers.append(worker)
        if cached is not None:
            cached.pins -= 1
        elif entry is not None and self.use_cache and req.key is not None and req.key not in self._cache:
            nb = self.ex.cache_bytes(req)
            if self._evict_for(nb):
                self._cache[req.key] = _Cached(entry, nb)
                self._cache_bytes += nb
        self._lock.notify_all()
