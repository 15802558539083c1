"""Scheduler logic of the serving engine on the CPU, against a timing-model
backend (no GPU): admission by HBM budget, arrival order, slot reuse,
back-pressure, rejection and error propagation."""
import pytest

from paper_2106_03452_amd.serve import Engine, MockBackend, Request, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def run(engine, reqs, clock, dt=1e-5, limit=10.0):
    """Advance a fake clock, submit each request at its arrival, step until idle."""
    pending = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    while (i < len(pending) or not engine.idle()) and clock.t < limit:
        while i < len(pending) and pending[i].arrival <= clock.t:
            engine.submit(pending[i])
            i += 1
        engine.step(clock.t)
        clock.t += dt
    assert clock.t < limit, "engine did not drain"


def make(n, res=64, bwd=False, gap=0.0, P=1000):
    return [Request(rid=i, res=res, npoints=P, backward=bwd, arrival=i * gap) for i in range(n)]


def test_all_requests_finish_and_latency_is_positive():
    clk = FakeClock()
    be = MockBackend(num_streams=2, clock=clk)
    eng = Engine(be, {64: 5000, 128: 5000}, hbm_budget=10 ** 12)
    reqs = make(20, 64, gap=1e-4) + [Request(100 + i, 128, 2000, True, 5e-5 + i * 2e-4) for i in range(10)]
    run(eng, reqs, clk)
    assert len(eng.finished) == 30 and not eng.rejected
    assert all(r.latency is not None and r.latency > 0 and r.error is None for r in eng.finished)
    st = latency_stats(eng.finished)
    assert st["n"] == 30 and st["p99_ms"] >= st["p50_ms"] > 0


def test_budget_limits_resident_slots_and_slots_are_reused():
    clk = FakeClock()
    be = MockBackend(num_streams=4, clock=clk)
    slot = be.slot_bytes(64, 1000)
    eng = Engine(be, {64: 1000}, hbm_budget=3 * slot, max_batch=8)
    run(eng, make(40, 64), clk)
    assert len(eng.finished) == 40
    assert be.allocated == 3 and eng.used == 3 * slot  # never more than the budget allows
    assert eng.classes[64].total == 3 and len(eng.classes[64].free) == 3


def test_arrival_order_within_a_class():
    clk = FakeClock()
    be = MockBackend(num_streams=1, clock=clk)
    slot = be.slot_bytes(64, 1000)
    eng = Engine(be, {64: 1000}, hbm_budget=2 * slot, max_batch=2)
    run(eng, make(12, 64, gap=1e-6), clk)
    starts = [r.start for r in sorted(eng.finished, key=lambda r: r.rid)]
    assert starts == sorted(starts)  # FIFO: an earlier request never starts after a later one


def test_blocked_class_does_not_block_others():
    clk = FakeClock()
    be = MockBackend(num_streams=2, clock=clk, cost=lambda res, bwd: 1e-2 if res == 256 else 1e-5)
    s256 = be.slot_bytes(256, 1000)
    s64 = be.slot_bytes(64, 1000)
    eng = Engine(be, {256: 1000, 64: 1000}, hbm_budget=2 * s256 + 2 * s64 + 1, max_batch=4)
    eng.per_class_budget = s256 + 1  # one 256 slot, a few 64 slots
    big = [Request(i, 256, 1000, False, 0.0) for i in range(3)]
    small = [Request(10 + i, 64, 1000, False, 1e-4) for i in range(4)]
    run(eng, big + small, clk, limit=1.0)
    t_small = max(r.done for r in eng.finished if r.res == 64)
    t_big_last = max(r.done for r in eng.finished if r.res == 256)
    assert t_small < t_big_last  # small requests passed the queued 256^3 ones


def test_rejects_unserved_requests():
    clk = FakeClock()
    eng = Engine(MockBackend(clock=clk), {64: 1000}, hbm_budget=10 ** 9)
    eng.submit(Request(0, 128, 10, False, 0.0))
    eng.submit(Request(1, 64, 5000, False, 0.0))
    eng.submit(Request(2, 64, 0, False, 0.0))
    assert len(eng.rejected) == 3 and eng.idle()
    assert all(r.error.startswith("rejected") for r in eng.rejected)


def test_allocation_failure_applies_back_pressure_not_failure():
    clk = FakeClock()
    be = MockBackend(num_streams=2, clock=clk, fail_alloc=2)  # only 2 slots can ever be allocated
    eng = Engine(be, {64: 1000}, hbm_budget=10 ** 12, max_batch=4)
    run(eng, make(10, 64), clk)
    assert len(eng.finished) == 10 and all(r.error is None for r in eng.finished)
    assert be.allocated == 2


def test_launch_failure_is_reported_per_request_and_engine_continues():
    clk = FakeClock()
    be = MockBackend(num_streams=1, clock=clk, fail_launch={2})
    eng = Engine(be, {64: 1000}, hbm_budget=be.slot_bytes(64, 1000), max_batch=1)
    run(eng, make(5, 64), clk)
    errs = [r for r in eng.finished if r.error]
    assert len(eng.finished) == 5 and len(errs) == 1 and "failure" in errs[0].error
