"""Continuous-batching reconstruction server on one GPU.

Requests (a geometry, measurements, penalty, lambda, iteration count) arrive at
any time.  A scheduler thread admits queued requests first-fit, in arrival
order, as soon as their device footprint fits the free part of the memory
budget and an execution slot is free; admitted solves run concurrently, one
HIP stream per slot, so requests that arrive while others are on the GPU join
them mid-flight.  Plans (FP64 tables, workspace, solver state) stay resident
in a pool keyed by geometry and mask and are reused; idle plans are evicted
least-recently-used when memory is needed.  Every request owns its plan while
it runs, and every kernel is deterministic, so a result is bitwise the same
alone and in the mix.

The executor is pluggable: HipExecutor drives liboct; tests drive the same
scheduler with an executor that needs no GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import hashlib
import threading
import time
from concurrent.futures import Future
from typing import Any, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    geom: Any                         # paper_2108_01438_amd.Geometry
    y: np.ndarray                     # measurements [batch][n_y][n_x][n_k], float32 (host)
    penalty: str = "l1"
    lam: float = 0.0                  # absolute regularisation weight
    iters: int = 50
    mask: Optional[np.ndarray] = None  # uint8 [n_y][n_x][n_k]
    delta: float = 0.0                # <= 0: from the plan's cached power iteration
    tv_inner: int = 10
    haar_levels: int = 3
    rid: int = -1
    arrival: float = 0.0
    admitted: float = 0.0
    finished: float = 0.0


class AdmissionError(RuntimeError):
    pass


class Server:
    """Admission by footprint + concurrent execution slots."""

    def __init__(self, executor, mem_budget: int, slots: int = 8, poll_s: float = 2e-4):
        self.ex = executor
        self.budget = int(mem_budget)
        self.slots = int(slots)
        self.poll_s = poll_s
        self._queue = collections.deque()
        self._running = {}
        self._lock = threading.Condition()
        self._stop = False
        self._next = 0
        self.used = 0
        self.completed = []
        self._thread = threading.Thread(target=self._loop, name="oct-server", daemon=True)
        self._thread.start()

    # ---- client side ------------------------------------------------------
    def submit(self, req: Request) -> Future:
        fut = Future()
        need = self.ex.footprint(req)
        with self._lock:
            req.rid = self._next
            self._next += 1
            req.arrival = time.perf_counter()
            if need > self.budget:
                fut.set_exception(AdmissionError(
                    f"request {req.rid} needs {need} B, more than the whole budget {self.budget} B"))
                return fut
            self._queue.append((req, fut, need))
            self._lock.notify()
        return fut

    def cancel(self, fut: Future) -> bool:
        """Cancel a request that has not been admitted yet."""
        with self._lock:
            for i, (r, f, n) in enumerate(self._queue):
                if f is fut:
                    del self._queue[i]
                    f.cancel()
                    return True
        return False

    def close(self, wait: bool = True):
        with self._lock:
            self._stop = True
            self._lock.notify()
        if wait:
            self._thread.join()
        self.ex.shutdown()

    # ---- scheduler --------------------------------------------------------
    def _admit(self):
        """First-fit in arrival order: admit every queued request that fits."""
        i = 0
        while i < len(self._queue) and len(self._running) < self.slots:
            req, fut, need = self._queue[i]
            free = self.budget - self.used - self.ex.cached_bytes()
            if need > free:
                self.ex.evict_idle(need - free)
                free = self.budget - self.used - self.ex.cached_bytes()
            if need <= free:
                del self._queue[i]
                self.used += need
                req.admitted = time.perf_counter()
                try:
                    handle = self.ex.start(req)
                except Exception as e:  # isolate the failure to this request
                    self.used -= need
                    fut.set_exception(e)
                    continue
                self._running[req.rid] = (req, fut, need, handle)
            else:
                i += 1

    def _reap(self):
        done = [rid for rid, (r, f, n, h) in self._running.items() if self.ex.done(h)]
        for rid in done:
            req, fut, need, h = self._running.pop(rid)
            try:
                out = self.ex.result(h)
                req.finished = time.perf_counter()
                fut.set_result(out)
                self.completed.append(req)
            except Exception as e:
                req.finished = time.perf_counter()
                fut.set_exception(e)
            finally:
                self.used -= need
        return bool(done)

    def _loop(self):
        while True:
            with self._lock:
                if self._stop and not self._queue and not self._running:
                    return
                self._admit()
                busy = bool(self._running)
                if not busy and not self._queue and not self._stop:
                    self._lock.wait(timeout=0.05)
                    continue
            reaped = self._reap() if busy else False
            if not reaped:
                time.sleep(self.poll_s)

    def latency_stats(self):
        lat = np.array([r.finished - r.arrival for r in self.completed])
        if lat.size == 0:
            return {}
        return {"n": int(lat.size), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean())}


def plan_footprint(P, geom) -> int:
    """Device bytes a pooled plan may hold over its life: plans are pooled by
    geometry and mask and keep every solver state they have allocated, so the
    bound covers every penalty (TV duals and the DT-CWT workspace together)."""
    return int(P.footprint_bytes(geom, -1))


def request_footprint(P, req: Request) -> int:
    """Admission size of a request: its plan's bound + the y and result buffers."""
    g = req.geom
    img = g.batch * g.n_y * g.n_x * g.n_depth * 8
    meas = g.batch * g.n_y * g.n_x * g.n_k * 4
    return plan_footprint(P, g) + img + meas


class HipExecutor:
    """Runs requests with liboct: one plan per in-flight request (pooled per
    geometry and mask), one stream and one launching thread per slot, device
    buffers for y and the result.  A solve issues a thousand or more kernel
    launches; they go out from the slot's own thread (ctypes releases the GIL
    during the call), so the scheduler thread never waits on a launch queue."""

    def __init__(self, slots: int = 8):
        import concurrent.futures as cf
        import torch
        import paper_2108_01438_amd as P
        self.P = P
        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free_streams = list(range(slots))
        self.idle = collections.OrderedDict()    # key -> list of idle plans (LRU order)
        self.lipschitz = {}                      # key -> L (power iteration, cached)
        self.plan_bytes = {}
        self._cached = 0                         # bytes held by idle plans
        self._lock = threading.Lock()            # pool, streams and caches
        self._workers = cf.ThreadPoolExecutor(max_workers=slots, thread_name_prefix="oct-slot")

    @staticmethod
    def key(req: Request):
        """Pool key: the geometry and a 256-bit digest of the mask (a plan is
        reused only for the same geometry and the same mask bytes)."""
        g = req.geom
        mk = None
        if req.mask is not None:
            mk = hashlib.blake2b(np.ascontiguousarray(req.mask, dtype=np.uint8).tobytes(), digest_size=32).digest()
        return (dataclasses.astuple(g), mk)

    def footprint(self, req: Request) -> int:
        return request_footprint(self.P, req)

    def cached_bytes(self) -> int:
        with self._lock:
            return self._cached

    def _plan(self, req: Request):
        k = self.key(req)
        with self._lock:
            lst = self.idle.get(k)
            if lst:
                plan = lst.pop()
                if not lst:
                    del self.idle[k]
                self._cached -= self.plan_bytes[id(plan)]
                return plan
        plan = self.P.Plan(req.geom, req.mask)   # outside the lock: host tables and uploads
        with self._lock:
            self.plan_bytes[id(plan)] = plan_footprint(self.P, req.geom)
        return plan

    def evict_idle(self, need: int) -> int:
        """Free idle plans, least recently used first, until `need` bytes are free."""
        freed = 0
        while freed < need:
            with self._lock:
                if not self.idle:
                    break
                k, lst = next(iter(self.idle.items()))
                plan = lst.pop()
                if not lst:
                    del self.idle[k]
                b = self.plan_bytes.pop(id(plan), 0)
                self._cached -= b
            freed += b
            plan.release()   # idle: its last solve's event has completed; no device-wide wait
        return freed

    def _run(self, req: Request, si: int):
        """The slot thread: plan, upload, solve, download, completion event."""
        torch = self.torch
        k = self.key(req)
        s = self.streams[si]
        plan = self._plan(req)
        try:
            if req.delta > 0:
                delta = req.delta
            else:
                with self._lock:
                    L = self.lipschitz.get(k)
                if L is None:
                    with torch.cuda.stream(s):
                        L = plan.lipschitz(50, stream=s)
                    with self._lock:
                        self.lipschitz[k] = L
                delta = 1.0 / (1.05 * L) if L > 0 else 1.0   # L = 0: nothing observed, any step
            with torch.cuda.stream(s):
                y = torch.from_numpy(np.ascontiguousarray(req.y, dtype=np.float32)).pin_memory().to(
                    "cuda", non_blocking=True)
                z, _ = plan.mbir_solve(y, req.penalty, req.lam, req.iters, delta=delta, tv_inner=req.tv_inner,
                                       haar_levels=req.haar_levels, stream=s)
                host = torch.empty(z.shape, dtype=z.dtype, pin_memory=True)
                host.copy_(z, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
        except Exception:
            self._release(k, plan)
            raise
        return {"ev": ev, "host": host, "keep": (y, z), "plan": plan, "key": k}

    def start(self, req: Request):
        with self._lock:
            si = self.free_streams.pop()
        return {"fut": self._workers.submit(self._run, req, si), "stream": si}

    def _release(self, k, plan):
        with self._lock:
            self.idle.setdefault(k, []).append(plan)
            self.idle.move_to_end(k)
            self._cached += self.plan_bytes[id(plan)]

    def done(self, h) -> bool:
        f = h["fut"]
        if not f.done():
            return False
        if f.exception() is not None:
            return True
        return f.result()["ev"].query()

    def result(self, h):
        try:
            r = h["fut"].result()
        finally:
            with self._lock:
                self.free_streams.append(h["stream"])
        r["ev"].synchronize()
        out = r["host"].numpy().copy()
        self._release(r["key"], r["plan"])
        r["keep"] = None
        return out

    def shutdown(self):
        self._workers.shutdown(wait=True)
        with self._lock:
            plans = [p for lst in self.idle.values() for p in lst]
            self.idle.clear()
            self._cached = 0
        for p in plans:
            p.release()


def run_sequential(executor, reqs):
    """Solve requests one at a time (the baseline); returns (outputs, seconds)."""
    outs = []
    t0 = time.perf_counter()
    for r in reqs:
        h = executor.start(r)
        while not executor.done(h):
            time.sleep(1e-4)
        outs.append(executor.result(h))
    return outs, time.perf_counter() - t0


__all__ = ["Request", "Server", "HipExecutor", "AdmissionError", "run_sequential", "plan_footprint",
           "request_footprint"]
