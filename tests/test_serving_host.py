"""Host-side logic of the serving loop, on the CPU with a mock clock (no GPU):

* admission -- FIFO waiting for a slot and for room in the particle budget, a
  request that does not fit does not block later ones, a departed human's slot
  is reused only after the in-flight work that uses it reports completion,
  departures of waiting humans;
* deadline accounting -- run_paced releases cycle c at t0 + c / rate, a
  cycle's latency is (completion seen by the host) - (release tick), the
  back-to-back polling while a cycle is in flight sees a completion within one
  poll, misses are latencies above the period, and arrivals/departures run
  after the tick inside the cycle's latency.
"""
import collections
import dataclasses

import numpy as np
import pytest

from paper_2603_01122_amd.serve import Admission, latency_summary, run_paced


@dataclasses.dataclass
class Req:
    hid: int
    N: int


class Flag:
    def __init__(self):
        self.done = False

    def query(self):
        return self.done


def test_admission_slots_budget_and_order():
    a = Admission(n_slots=2, budget=100)
    for hid, n in [(1, 60), (2, 50), (3, 30), (4, 10)]:
        a.submit(Req(hid, n))
    got = a.admit()
    # 1 fits (60); 2 would exceed the budget and waits; 3 fits (90); no slot left for 4
    assert [(s, r.hid) for s, r in got] == [(0, 1), (1, 3)]
    assert [r.hid for r in a.waiting] == [2, 4]
    assert a.in_use == 90
    assert a.admit() == []                       # nothing changed
    # 1 leaves with no work in flight: its slot is free at once; 2 still does not
    # fit (30 + 50 <= 100 does), so 2 is admitted before 4 (FIFO)
    assert a.depart(1) == 0
    got = a.admit()
    assert [(s, r.hid) for s, r in got] == [(0, 2)]
    assert a.in_use == 80 and [r.hid for r in a.waiting] == [4]
    # a waiting human can leave the queue
    assert a.depart(4) is None
    assert not a.waiting
    assert set(a.active) == {2, 3}


def test_departed_slot_waits_for_in_flight_work():
    a = Admission(n_slots=1)
    a.submit(Req(7, 10))
    assert [s for s, _ in a.admit()] == [0]
    f1, f2 = Flag(), Flag()
    assert a.depart(7, busy=[f1, f2]) == 0
    a.submit(Req(8, 10))
    assert a.admit() == []                       # slot 0 still used by cycles in flight
    f1.done = True
    assert a.admit() == []
    f2.done = True
    got = a.admit()
    assert [(s, r.hid) for s, r in got] == [(0, 8)]
    assert a.in_use == 10


def test_unlimited_budget_and_many_slots():
    a = Admission(n_slots=3)
    for hid in range(5):
        a.submit(Req(hid, 10 ** 9))
    assert [r.hid for _, r in a.admit()] == [0, 1, 2]
    assert [r.hid for r in a.waiting] == [3, 4]


class MockClock:
    """Reading the clock costs 1 us (the loop spins on it in the last 200 us
    before a tick)."""

    def __init__(self):
        self.t = 100.0

    def __call__(self):
        self.t += 1e-6
        return self.t

    def sleep(self, dt):
        assert dt > 0
        self.t += dt


@dataclasses.dataclass
class Rec:
    cycle: int
    release: float
    done_at: float
    completed: float = None

    @property
    def latency(self):
        return None if self.completed is None else self.completed - self.release


class MockServer:
    """Cycle c takes service[c] seconds of device time after it is launched
    (or after the previous cycle finishes, whichever is later)."""

    def __init__(self, clock, service, host_cost=0.0):
        self.clock, self.service, self.host_cost = clock, service, host_cost
        self.pending = collections.deque()
        self.launched = []
        self.recs = []
        self.busy_until = 0.0

    def step(self, obs, release=None):
        c = len(self.launched)
        self.clock.t += self.host_cost
        start = max(self.clock(), self.busy_until)
        self.busy_until = start + self.service[c]
        r = Rec(c, release, self.busy_until)
        self.launched.append((c, release, self.clock(), obs))
        self.pending.append(r)
        self.recs.append(r)
        return r

    def poll(self):
        now = self.clock()
        while self.pending and self.pending[0].done_at <= now:
            self.pending.popleft().completed = now
        return len(self.pending)

    def drain(self):
        while self.poll():
            self.clock.sleep(20e-6)


def test_paced_latency_and_misses_with_mock_clock():
    clk = MockClock()
    rate = 125.0
    period = 1.0 / rate
    service = [1.0e-3] * 50
    service[10] = 9.0e-3                         # one slow cycle misses its deadline
    service[30] = 7.5e-3                         # a long one that still makes it
    srv = MockServer(clk, service, host_cost=30e-6)
    events = []
    lat = run_paced(srv, lambda c: {0: (float(c), 0.0)}, len(service), rate,
                    before_step=lambda c: events.append((c, clk())), clock=clk,
                    sleep=clk.sleep)
    assert lat.shape == (50,)
    rel0 = srv.launched[0][1]
    for c, (cc, release, t_launch, obs) in enumerate(srv.launched):
        assert cc == c and obs == {0: (float(c), 0.0)}
        assert release == pytest.approx(rel0 + c * period, abs=1e-12)
        # arrivals/departures run after the tick, before the launch
        assert release <= events[c][1] <= t_launch
    for c, r in enumerate(srv.recs):
        # the device finishes service[c] after the launch (or after cycle 10,
        # for the cycle queued behind it); the host sees it within one poll
        busy_wait = service[10] - period if c == 11 else 0.0
        finish = r.done_at - r.release
        assert 30e-6 + busy_wait + service[c] <= finish <= 30e-6 + busy_wait + service[c] + 10e-6
        # while a cycle is in flight the loop polls back to back: the host
        # sees the completion within one poll (two clock reads here); the last
        # cycle completes in the final drain, which polls every 20 us
        slack = 5e-6 if c < len(service) - 1 else 25e-6
        assert finish <= lat[c] <= finish + slack, (c, lat[c], finish)
    s = latency_summary(lat, period)
    assert s["deadline_misses"] == 1 and s["cycles"] == 50
    assert abs(s["max_ms"] - lat.max() * 1e3) < 1e-3
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3, abs=1e-3)


def test_latency_summary_counts_misses_strictly_above_the_period():
    period = 8e-3
    s = latency_summary([1e-3, 8e-3, 8.0001e-3, 2e-3], period)
    assert s["deadline_misses"] == 1
    assert s["deadline_ms"] == 8.0 and s["cycles"] == 4
