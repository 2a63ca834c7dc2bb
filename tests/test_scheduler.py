"""The serving policy on the CPU: fake executor with scripted durations and
a simulated clock."""
import math

import pytest

from paper_2504_17987_amd.serve import ClassSpec, FakeExecutor, Request, Scheduler, poisson_trace


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def simulate(sched, clock, trace, dt=1e-5, limit=10.0):
    i = 0
    while i < len(trace) or sched.pending():
        assert clock.t < limit, "simulation did not drain"
        while i < len(trace) and trace[i].arrival <= clock.t:
            sched.submit(trace[i])
            i += 1
        sched.step(clock.t)
        clock.t += dt


CLASSES = [ClassSpec("s", 512, 512, 16, 10_000, 1_000),
           ClassSpec("m", 1024, 1024, 8, 40_000, 4_000),
           ClassSpec("l", 2048, 2048, 4, 160_000, 16_000)]


def make(budget=10**9, max_wait=2e-3, inflight=2, dur=None):
    clock = Clock()
    dur = dur or (lambda cls, n: {"s": 1e-4, "m": 2e-4, "l": 6e-4}[cls] * (1 + 0.1 * n))
    ex = FakeExecutor(dur, clock)
    return Scheduler(CLASSES, ex, budget, max_wait=max_wait, inflight=inflight), ex, clock


def test_all_requests_complete_fifo_within_class():
    sched, ex, clock = make()
    streams = [(s, "sml"[s % 3]) for s in range(12)]
    for s, c in streams:
        assert sched.admit(s, c)
    trace = poisson_trace(streams, 250.0, 0.5, 16, seed=1)
    simulate(sched, clock, trace)
    assert len(sched.finished) == len(trace)
    assert all(not math.isnan(r.done) and r.done >= r.start >= r.arrival for r in trace)
    for c in "sml":
        starts = [(r.arrival, r.start) for r in trace if r.cls == c]
        # FIFO: a later arrival never starts before an earlier one of its class
        s_sorted = [s for _, s in sorted(starts)]
        assert all(a <= b for a, b in zip(s_sorted, s_sorted[1:]))


def test_batches_fill_and_respect_capacity():
    sched, ex, clock = make(max_wait=1.0, dur=lambda c, n: 5e-3)
    sched.admit(0, "s")
    # a burst of 40 requests at t=0: batches of 16, 16 (two in flight), then 8
    trace = [Request(i, 0, "s", i % 16, 0.0) for i in range(40)]
    simulate(sched, clock, trace)
    sizes = [n for c, n, t in ex.log]
    assert sizes[:2] == [16, 16] and sum(sizes) == 40 and max(sizes) <= 16


def test_max_wait_bounds_latency_under_light_load():
    sched, ex, clock = make(max_wait=2e-3, dur=lambda c, n: 1e-4)
    sched.admit(0, "l")
    trace = [Request(i, 0, "l", 0, 0.01 * i) for i in range(20)]
    simulate(sched, clock, trace)
    # device idle on every arrival: each request launches at once
    assert max(r.start - r.arrival for r in trace) < 2e-5


def test_no_starvation_under_overload():
    # the large class is slow; small requests keep flowing
    sched, ex, clock = make(max_wait=1e-3, dur=lambda c, n: 2e-3 if c == "l" else 2e-4, inflight=1)
    streams = [(0, "s"), (1, "l")]
    for s, c in streams:
        sched.admit(s, c)
    trace = poisson_trace(streams, 2000.0, 0.2, 4, seed=3)
    simulate(sched, clock, trace)
    small = [r.done - r.arrival for r in trace if r.cls == "s"]
    large = [r.done - r.arrival for r in trace if r.cls == "l"]
    assert len(sched.finished) == len(trace)
    assert max(small) < 0.01 and max(large) < 0.2


def test_admission_respects_budget_and_releases():
    # budget for the small class (2 runners) and 2 of its streams only
    budget = 2 * 10_000 + 2 * 1_000
    sched, ex, clock = make(budget=budget)
    assert sched.admit(0, "s") and sched.admit(1, "s")
    assert not sched.admit(2, "s")                 # does not fit: waits
    assert not sched.admit(3, "m")
    assert sched.used <= budget
    assert not sched.submit(Request(0, 2, "s", 0, 0.0))   # not admitted yet
    sched.retire(0)                                # frees one stream's bytes
    assert 2 in sched.admitted and 3 not in sched.admitted
    assert sched.used <= budget
    sched.retire(1)
    sched.retire(2)                                # class s empties: its runners are released
    assert sched.used == 0
    assert 3 not in sched.admitted                 # its class alone exceeds the budget: still waiting
    sched.set_budget(2 * 40_000 + 4_000)           # more memory: waiting streams are re-tried
    assert 3 in sched.admitted and sched.used == sched.budget


def test_idle_class_launches_while_another_class_runs():
    # a long batch of the large class is on the device; a small request that
    # arrives meanwhile starts at once instead of waiting for max_wait
    sched, ex, clock = make(max_wait=1.0, dur=lambda c, n: 5e-3 if c == "l" else 1e-4)
    sched.admit(0, "l")
    sched.admit(1, "s")
    trace = [Request(0, 0, "l", 0, 0.0), Request(1, 1, "s", 0, 1e-3)]
    simulate(sched, clock, trace)
    assert trace[1].start - trace[1].arrival < 2e-5


class HookedExecutor(FakeExecutor):
    def __init__(self, *a):
        super().__init__(*a)
        self.events = []

    def class_admitted(self, cls):
        self.events.append(("admit", cls))

    def class_retired(self, cls):
        self.events.append(("retire", cls))


def test_runners_follow_admission_and_refused_requests_are_counted_apart():
    """A class's runners are built when its first stream is admitted and
    released when its last stream retires; requests of a refused stream are
    listed apart and kept out of the latency statistics."""
    from paper_2504_17987_amd.serve import latency_stats
    clock = Clock()
    ex = HookedExecutor(lambda cls, n: 1e-4, clock)
    # budget: class s (2 runners + streams) fits, class l does not
    budget = 2 * 10_000 + 2 * 1_000
    sched = Scheduler(CLASSES, ex, budget, inflight=2)
    assert sched.admit(0, "s") and sched.admit(1, "s")
    assert not sched.admit(2, "l")
    assert ex.events == [("admit", "s")]
    trace = poisson_trace([(0, "s"), (1, "s"), (2, "l")], 500.0, 0.05, 2, seed=3)
    simulate(sched, clock, trace)
    refused = [r for r in trace if r.stream == 2]
    assert refused and sched.refused == refused
    st = latency_stats(trace)
    assert st["refused"] == len(refused) and st["n"] == len(trace) - len(refused)
    assert math.isfinite(st["p99_ms"])
    sched.retire(0)
    assert ("retire", "s") not in ex.events
    sched.retire(1)
    assert ex.events[-1] == ("retire", "s")
    # the budget freed by class s admits the waiting l stream, whose runners are then built
    sched.set_budget(budget + 160_000 * 2 + 16_000)
    assert sched.admitted.get(2) == "l" and ex.events[-1] == ("admit", "l")
