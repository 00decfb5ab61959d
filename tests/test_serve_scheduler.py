"""Admission logic of the serving loop, on the CPU with a fake clock and a fake engine."""
import pytest

from paper_2010_08581_amd.serve import Scheduler, run, summarize


class FakeClock:
    """Advances by a fixed tick on every read, so a spinning loop makes progress."""

    def __init__(self, tick=1e-4):
        self.t = 0.0
        self.tick = tick

    def __call__(self):
        self.t += self.tick
        return self.t

    def wait(self, dt):
        if dt > 0:
            self.t += dt


class FakeEngine:
    """Job of request r runs for r["dur"] seconds of the fake clock; footprint r["mem"]."""

    def __init__(self, clock, fail_ids=()):
        self.clock = clock
        self.fail_ids = set(fail_ids)
        self.started = []  # (id, slot, time)
        self.active = set()
        self.max_active = 0

    def footprint(self, req):
        return req["mem"]

    def start(self, req, slot):
        assert slot not in {s for (_, s) in self.active}, "slot handed out twice"
        self.started.append((req["id"], slot, self.clock.t))
        self.active.add((req["id"], slot))
        self.max_active = max(self.max_active, len(self.active))
        return dict(req=req, slot=slot, end=self.clock.t + req["dur"])

    def poll(self, job):
        if self.clock.t < job["end"]:
            return False
        if job["req"]["id"] in self.fail_ids:
            raise RuntimeError("solve failed")
        return True

    def finish(self, job):
        self.active.discard((job["req"]["id"], job["slot"]))
        return dict(fit=0.01 * (1 + job["req"]["id"]))

    def abandon(self, job):
        self.active.discard((job["req"]["id"], job["slot"]))


def req(i, arrival=0.0, dur=0.01, mem=1, dims=(8, 8, 8), samples=16, sweeps=2):
    return dict(id=i, arrival=arrival, dur=dur, mem=mem, dims=list(dims), ranks=[2] * len(dims),
                samples=samples, sweeps=sweeps, seed=0)


def test_slots_bound_concurrency_and_all_finish():
    clk = FakeClock()
    eng = FakeEngine(clk)
    reqs = [req(i) for i in range(7)]
    res, wall, sched = run(eng, reqs, slots=3, mem_budget=100, clock=clk, wait=clk.wait)
    assert [r.id for r in res] == list(range(7))
    assert all(r.error is None for r in res)
    assert eng.max_active == 3 and sched.peak_running == 3
    # FIFO: admission order follows arrival (then id)
    assert [s[0] for s in eng.started] == list(range(7))
    # the first three start at once; the fourth only after one of them finished
    t_first = [s[2] for s in eng.started[:3]]
    assert max(t_first) < 0.005
    assert eng.started[3][2] >= 0.01
    assert sched.mem_in_use == 0 and not sched.running


def test_memory_budget_limits_admission():
    clk = FakeClock()
    eng = FakeEngine(clk)
    reqs = [req(i, mem=40) for i in range(5)]
    res, wall, sched = run(eng, reqs, slots=8, mem_budget=100, clock=clk, wait=clk.wait)
    assert all(r.error is None for r in res)
    assert eng.max_active == 2  # 3 x 40 > 100
    assert sched.peak_mem == 80


def test_over_budget_request_refused_others_served():
    clk = FakeClock()
    eng = FakeEngine(clk)
    reqs = [req(0, mem=10), req(1, mem=1000), req(2, mem=10)]
    res, wall, sched = run(eng, reqs, slots=2, mem_budget=100, clock=clk, wait=clk.wait)
    assert res[1].error is not None and "budget" in res[1].error and res[1].admitted is None
    assert res[0].error is None and res[2].error is None
    assert [s[0] for s in eng.started] == [0, 2]


def test_head_of_line_waits_for_memory_in_order():
    clk = FakeClock()
    eng = FakeEngine(clk)
    # request 1 needs most of the budget: request 2 (small) must not overtake it
    reqs = [req(0, mem=60, dur=0.02), req(1, mem=90, arrival=0.001), req(2, mem=5, arrival=0.002)]
    res, wall, sched = run(eng, reqs, slots=4, mem_budget=100, clock=clk, wait=clk.wait)
    order = [s[0] for s in eng.started]
    assert order == [0, 1, 2]
    t = {s[0]: s[2] for s in eng.started}
    assert t[1] >= 0.02  # waited for request 0's memory
    assert res[1].admitted >= 0.02


def test_failed_request_isolated():
    clk = FakeClock()
    eng = FakeEngine(clk, fail_ids={1})
    reqs = [req(i) for i in range(4)]
    res, wall, sched = run(eng, reqs, slots=2, mem_budget=100, clock=clk, wait=clk.wait)
    assert res[1].error is not None and "solve failed" in res[1].error
    assert all(res[i].error is None for i in (0, 2, 3))
    assert not eng.active and sched.mem_in_use == 0


def test_arrivals_over_time_and_latency():
    clk = FakeClock()
    eng = FakeEngine(clk)
    # arrivals 50 ms apart, each job 10 ms: never queued, latency ~ job time
    reqs = [req(i, arrival=0.05 * i, dur=0.01) for i in range(5)]
    res, wall, sched = run(eng, reqs, slots=1, mem_budget=100, clock=clk, wait=clk.wait)
    for r in res:
        assert r.admitted - r.arrival < 0.002
        assert 0.01 <= r.latency < 0.012
    s = summarize(res, wall)
    assert s["completed"] == 5 and s["failed"] == 0
    assert 10.0 <= s["p50_ms"] <= s["p99_ms"] < 12.0
    assert s["rows_per_s"] == pytest.approx(5 * 16 * 3 * 2 / wall)


def test_scheduler_rejects_bad_configuration():
    with pytest.raises(ValueError):
        Scheduler(FakeEngine(FakeClock()), slots=0, mem_budget=10)
    with pytest.raises(ValueError):
        Scheduler(FakeEngine(FakeClock()), slots=1, mem_budget=0)
