"""Scheduler of the serving loop on the CPU with an executor that needs no GPU:
admission by footprint, mid-flight admission, first-fit, rejection,
cancellation and error isolation."""
import threading
import time

import numpy as np
import pytest

from paper_2108_01438_amd.serve import AdmissionError, Request, Server


class FakeExecutor:
    """Each request 'runs' for a time proportional to its footprint."""

    def __init__(self, bytes_per_s=1e9, fail=()):
        self.rate = bytes_per_s
        self.fail = set(fail)
        self.running = 0
        self.max_running = 0
        self.lock = threading.Lock()

    def footprint(self, req):
        return int(req.y.nbytes)

    def cached_bytes(self):
        return 0

    def evict_idle(self, need):
        return 0

    def start(self, req):
        if req.rid in self.fail:
            raise RuntimeError(f"injected failure for {req.rid}")
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
        return {"t_end": time.perf_counter() + self.footprint(req) / self.rate, "out": float(req.y.sum())}

    def done(self, h):
        return time.perf_counter() >= h["t_end"]

    def result(self, h):
        with self.lock:
            self.running -= 1
        return h["out"]

    def shutdown(self):
        pass


def req(nbytes, val=1.0):
    return Request(geom=None, y=np.full(nbytes // 4, val, dtype=np.float32))


def test_all_complete_with_own_results():
    ex = FakeExecutor(bytes_per_s=1e8)
    srv = Server(ex, mem_budget=10_000_000, slots=4)
    futs = [srv.submit(req(400_000, v)) for v in range(1, 9)]
    outs = [f.result(timeout=10) for f in futs]
    srv.close()
    assert outs == [100_000.0 * v for v in range(1, 9)]
    st = srv.latency_stats()
    assert st["n"] == 8 and st["p99_s"] >= st["p50_s"] > 0


def test_admission_respects_memory_budget():
    ex = FakeExecutor(bytes_per_s=2e7)
    srv = Server(ex, mem_budget=2_500_000, slots=8)
    futs = [srv.submit(req(1_000_000)) for _ in range(6)]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert ex.max_running == 2          # two 1 MB requests fit a 2.5 MB budget, three do not


def test_slots_limit_concurrency():
    ex = FakeExecutor(bytes_per_s=2e7)
    srv = Server(ex, mem_budget=10**9, slots=3)
    futs = [srv.submit(req(200_000)) for _ in range(9)]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert ex.max_running == 3


def test_mid_flight_admission():
    """A request arriving while another runs is admitted before that one ends."""
    ex = FakeExecutor(bytes_per_s=1e7)
    srv = Server(ex, mem_budget=10**8, slots=4)
    fa = srv.submit(req(2_000_000))        # ~0.2 s
    time.sleep(0.05)
    fb = srv.submit(req(100_000))
    fa.result(timeout=10)
    fb.result(timeout=10)
    srv.close()
    a, b = sorted(srv.completed, key=lambda r: r.rid)
    assert b.admitted < a.finished
    assert b.finished < a.finished


def test_first_fit_passes_a_blocked_request():
    ex = FakeExecutor(bytes_per_s=1e7)
    srv = Server(ex, mem_budget=3_000_000, slots=4)
    f1 = srv.submit(req(2_000_000))        # runs
    time.sleep(0.02)
    f2 = srv.submit(req(2_000_000))        # waits for memory
    f3 = srv.submit(req(500_000))          # fits now: admitted ahead of f2
    for f in (f1, f2, f3):
        f.result(timeout=10)
    srv.close()
    r = {x.rid: x for x in srv.completed}
    assert r[2].admitted < r[1].admitted


def test_oversized_request_rejected_others_served():
    ex = FakeExecutor()
    srv = Server(ex, mem_budget=1_000_000, slots=2)
    big = srv.submit(req(4_000_000))
    ok = srv.submit(req(100_000))
    with pytest.raises(AdmissionError):
        big.result(timeout=5)
    assert ok.result(timeout=5) == 25_000.0
    srv.close()


def test_failure_is_isolated():
    ex = FakeExecutor(bytes_per_s=1e8, fail={1})
    srv = Server(ex, mem_budget=10**8, slots=2)
    futs = [srv.submit(req(100_000)) for _ in range(4)]
    with pytest.raises(RuntimeError, match="injected"):
        futs[1].result(timeout=5)
    assert [futs[i].result(timeout=5) for i in (0, 2, 3)] == [25_000.0] * 3
    srv.close()
    assert srv.used == 0


def test_cancel_queued_request():
    ex = FakeExecutor(bytes_per_s=1e7)
    srv = Server(ex, mem_budget=1_500_000, slots=1)
    f1 = srv.submit(req(1_000_000))
    f2 = srv.submit(req(1_000_000))
    assert srv.cancel(f2)
    assert f2.cancelled()
    f1.result(timeout=10)
    srv.close()
    assert len(srv.completed) == 1


def test_serving_mix_geometries_pass_plan_validation():
    """Every geometry the serving mix draws (7-smooth sizes, some with radix-7
    and many radix-3 butterflies per stage) passes the plan's shape checks.
    Without a GPU a valid plan stops at the device query (status 3); a shape
    the kernels do not support would stop earlier with status 4."""
    import paper_2108_01438_amd as P
    import synth
    seen = set()
    for seed in (4, 5, 6):
        for spec in synth.serving_mix(np.random.default_rng(seed), 200):
            key = tuple(sorted(spec["geom"].items()))
            if key in seen:
                continue
            seen.add(key)
            geo = dict(synth.OPTICS)
            geo.update(spec["geom"])
            try:
                P.Plan(P.Geometry.from_dict(geo)).close()
            except P.OctError as e:
                assert e.status != 4, (spec["geom"], str(e))
    assert len(seen) > 100


def test_admission_footprint_covers_every_penalty_state():
    """A pooled plan keeps every solver state it allocates (plans are pooled
    by geometry and mask, not penalty), so admission and pool accounting use a
    bound that covers them all: at least the library's footprint for TV and
    for the DT-CWT (whose volume workspace is the largest), for B-scans and
    volumes, plus the request's own y and result buffers."""
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.serve import Request, plan_footprint, request_footprint
    for geo in (P.Geometry(n_depth=1024, n_x=512, n_k=1024),
                P.Geometry(n_depth=1024, n_x=64, n_y=64, n_k=1024, lateral_dims=2)):
        img = geo.n_y * geo.n_x * geo.n_depth * 8
        meas = geo.n_y * geo.n_x * geo.n_k * 4
        tv = P.footprint_bytes(geo, P.PEN_TV)
        dt = P.footprint_bytes(geo, P.PEN_DTCWT)
        both = plan_footprint(P, geo)
        assert both >= max(tv, dt)
        # both states together: the DT-CWT workspace on top of the TV footprint
        extra_dt = dt - P.footprint_bytes(geo, P.PEN_L1)
        assert both >= tv + extra_dt
        r = Request(geom=geo, y=np.zeros((1, geo.n_y, geo.n_x, geo.n_k), np.float32), penalty="dtcwt")
        assert request_footprint(P, r) == both + img + meas
    v = P.Geometry(n_depth=1024, n_x=64, n_y=64, n_k=1024, lateral_dims=2)
    n = 64 * 64 * 1024
    assert P.footprint_bytes(v, P.PEN_DTCWT) - P.footprint_bytes(v, P.PEN_L1) == 24 * 8 * n
