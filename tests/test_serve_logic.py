"""Host logic of the serving loop (no GPU): trace generation, FIFO admission
under an HBM budget, tick planning without overshoot, and the latency
summary, driven by a simulated clock and executor."""
import math

import numpy as np
import pytest

from paper_2303_10785_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Each group runs on a lane of its own (groups overlap fully); a launch
    of k steps finishes after a fixed time per cell-step of its members.
    Counts the steps each request gets."""

    def __init__(self, clock, sec_per_cell_step=1e-9, bytes_per_cell=100):
        self.clock = clock
        self.cost = sec_per_cell_step
        self.bpc = bytes_per_cell
        self.live = {}
        self.steps = {}
        self.admitted = []
        self.max_live_bytes = 0
        self.finish = {}
        self.launch_log = []
        self.max_concurrent = 0

    def bytes_of(self, r):
        return self.bpc * r.ncell

    def admit(self, r):
        self.live[r.rid] = r
        self.steps[r.rid] = 0
        self.admitted.append(r.rid)
        self.max_live_bytes = max(self.max_live_bytes, sum(self.bytes_of(x) for x in self.live.values()))

    def launch(self, group, rids, k):
        assert self.done(group), "a group is relaunched only when idle"
        assert rids and all(self.live[rid].group == group for rid in rids)
        for rid in rids:
            self.steps[rid] += k
        self.finish[group] = self.clock.t + self.cost * k * sum(self.live[rid].ncell for rid in rids)
        self.launch_log.append((self.clock.t, group, tuple(sorted(rids)), k))
        busy = sum(1 for f in self.finish.values() if f > self.clock.t)
        self.max_concurrent = max(self.max_concurrent, busy)

    def done(self, group):
        return self.clock.t >= self.finish.get(group, 0.0)

    def retire(self, r):
        assert self.steps[r.rid] == r.steps
        assert self.done(r.group)
        del self.live[r.rid]
        return True


def test_trace_statistics():
    tr = serve.make_trace(4000, rate=50.0, seed=1)
    gaps = np.diff([0.0] + [r.arrival for r in tr])
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0
    two = [r for r in tr if r.ndim == 2]
    three = [r for r in tr if r.ndim == 3]
    assert 0.45 < len(two) / len(tr) < 0.55
    assert min(r.n for r in two) >= 64 and max(r.n for r in two) <= 1024
    assert min(r.n for r in three) >= 64 and max(r.n for r in three) <= 256
    assert min(r.steps for r in tr) >= 20 and max(r.steps for r in tr) <= 500
    # log-uniform sizes: median near the geometric mean of the range
    assert abs(math.log(np.median([r.n for r in two])) - 0.5 * math.log(64 * 1024)) < 0.15
    assert {r.ic for r in two} == {"vortex", "sod"} and {r.ic for r in three} == {"column"}
    assert 0.45 < np.mean([r.precision == "fp32_bulk" for r in tr]) < 0.55
    assert [r.arrival for r in serve.make_trace(50, seed=1)] == [r.arrival for r in tr[:50]]
    fast = serve.rescale(tr[:10], 2.0)
    assert [r.arrival for r in fast] == [r.arrival / 2.0 for r in tr[:10]]


def test_fifo_admission_respects_budget():
    clock = Clock()
    ex = FakeExecutor(clock, sec_per_cell_step=1e-6, bytes_per_cell=1)
    reqs = [serve.Request(i, 0.001 * i, 2, 100, 10, "fp64", "vortex", i) for i in range(5)]
    budget = 2 * 100 * 100  # two requests at a time
    out = serve.run(reqs, ex, budget, clock=clock, sleep=clock.sleep)
    assert out["requests"] == 5
    assert ex.max_live_bytes <= budget
    assert ex.admitted == [0, 1, 2, 3, 4]  # arrival order
    assert all(v == 10 for v in ex.steps.values())


def test_head_of_line_request_waits_for_room():
    clock = Clock()
    ex = FakeExecutor(clock, sec_per_cell_step=1e-6, bytes_per_cell=1)
    big = serve.Request(1, 0.01, 3, 20, 30, "fp64", "column", 1)       # 8000 B
    small = serve.Request(2, 0.02, 2, 10, 5, "fp64", "vortex", 2)      # 100 B
    first = serve.Request(0, 0.0, 2, 80, 40, "fp32_bulk", "sod", 0)    # 6400 B
    out = serve.run([first, big, small], ex, 9000, clock=clock, sleep=clock.sleep)
    assert out["requests"] == 3
    # FIFO: the small request does not pass the big one that is waiting
    assert ex.admitted == [0, 1, 2]
    assert big.admitted >= first.done
    assert small.admitted >= big.admitted


def test_request_larger_than_budget_is_rejected():
    clock = Clock()
    ex = FakeExecutor(clock)
    with pytest.raises(ValueError):
        serve.run([serve.Request(0, 0.0, 3, 100, 10, "fp64", "column", 0)], ex, 1000,
                  clock=clock, sleep=clock.sleep)


def test_groups_advance_without_overshoot_and_stats():
    clock = Clock()
    ex = FakeExecutor(clock, sec_per_cell_step=1e-8)
    tr = serve.make_trace(60, rate=200.0, seed=3, n2d=(8, 32), n3d=(4, 8), steps=(3, 60))
    out = serve.run(tr, ex, 10 ** 12, tick_steps=7, clock=clock, sleep=clock.sleep)
    assert out["requests"] == 60
    assert all(ex.steps[r.rid] == r.steps for r in tr)
    lat = sorted(r.done - r.arrival for r in tr)
    assert out["latency_p50_s"] == pytest.approx(float(np.percentile(lat, 50)))
    assert out["latency_p99_s"] == pytest.approx(float(np.percentile(lat, 99)))
    assert out["latency_p99_s"] >= out["latency_p50_s"] > 0
    work = sum(r.work for r in tr)
    assert out["achieved_cell_updates_per_s"] == pytest.approx(work / out["makespan_s"])
    assert all(r.admitted >= r.arrival and r.done > r.admitted for r in tr)


def test_plan_takes_smallest_remaining_per_group():
    s = serve.Scheduler(10 ** 9, lambda r: 1, tick_steps=25)
    reqs = [serve.Request(0, 0, 2, 8, 40, "fp64", "vortex", 0),
            serve.Request(1, 0, 2, 8, 12, "fp64", "sod", 1),
            serve.Request(2, 0, 2, 8, 90, "fp32_bulk", "vortex", 2),
            serve.Request(3, 0, 3, 8, 5, "fp64", "column", 3)]
    for r in reqs:
        s.arrive(r)
    s.admit(0.0)
    assert s.plan() == {("2d", "fp64"): (12, [0, 1]), ("2d", "fp32_bulk"): (25, [2]), ("3d", 3): (5, [3])}
    assert s.plan(busy={("2d", "fp64"): None}) == {("2d", "fp32_bulk"): (25, [2]), ("3d", 3): (5, [3])}
    done = s.advanced([0, 1], 12, 1.0)
    assert [r.rid for r in done] == [1]
    assert s.plan()[("2d", "fp64")] == (25, [0])


def test_groups_overlap_and_late_arrivals_join_at_the_next_launch():
    """A long 3-D request does not hold up 2-D work: groups run
    concurrently. A 2-D request arriving while its batch is in flight joins
    at the batch's next launch, and the in-flight launch does not count
    steps for it."""
    clock = Clock()
    ex = FakeExecutor(clock, sec_per_cell_step=1e-6, bytes_per_cell=1)
    slow3d = serve.Request(0, 0.0, 3, 20, 50, "fp64", "column", 0)     # 8000 cells x 50 steps
    a = serve.Request(1, 0.0, 2, 30, 40, "fp64", "vortex", 1)          # 9 ms per 10-step launch
    b = serve.Request(2, 0.005, 2, 30, 20, "fp64", "sod", 2)
    out = serve.run([slow3d, a, b], ex, 10 ** 9, tick_steps=10, clock=clock, sleep=clock.sleep)
    assert out["requests"] == 3 and all(ex.steps[r.rid] == r.steps for r in (slow3d, a, b))
    assert ex.max_concurrent >= 2
    # the 2-D requests finish long before the 3-D one
    assert a.done < slow3d.done and b.done < slow3d.done
    # b was admitted during a's first launch and first ran with it afterwards
    first_a = [x for x in ex.launch_log if x[1] == ("2d", "fp64")][0]
    assert first_a[2] == (1,)
    joint = [x for x in ex.launch_log if x[2] == (1, 2)]
    assert joint and joint[0][0] >= b.admitted
