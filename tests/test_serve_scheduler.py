"""Host-side checks of the serving scheduler (no GPU): a fake executor with
service times on a mock clock stands in for the device."""

import random

import pytest

from paper_1908_06096_amd.serve import Request, Scheduler, percentile


class MockClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-3):
        self.t += dt


class FakeExecutor:
    """Tables cost table_bytes per (N, prec); a request's buffers cost
    fields * unit; service time proportional to N * fields."""

    def __init__(self, clock, table_bytes=100, unit=10):
        self.clock = clock
        self.table_bytes = table_bytes
        self.unit = unit
        self.tables = {}
        self.busy = {}
        self.buf = 0
        self.evicted = []
        self.launched = []

    def footprint(self, req):
        key = (req.truncation, req.precision)
        return req.fields * self.unit + (0 if key in self.tables else self.table_bytes)

    def resident(self):
        return len(self.tables) * self.table_bytes + self.buf

    def inflight(self):
        return self.buf

    def evictable(self):
        return sum(self.table_bytes for k in self.tables if self.busy.get(k, 0) == 0)

    def evict(self, nbytes):
        freed = 0
        for k in list(self.tables):
            if freed >= nbytes:
                break
            if self.busy.get(k, 0):
                continue
            del self.tables[k]
            self.evicted.append(k)
            freed += self.table_bytes
        return freed

    def launch(self, req, slot):
        key = (req.truncation, req.precision)
        self.tables[key] = True
        self.busy[key] = self.busy.get(key, 0) + 1
        self.buf += req.fields * self.unit
        self.launched.append(req.rid)
        return (req, self.clock() + 1e-4 * req.truncation * req.fields)

    def done(self, h):
        return self.clock() >= h[1]

    def finish(self, h):
        req = h[0]
        key = (req.truncation, req.precision)
        self.busy[key] -= 1
        self.buf -= req.fields * self.unit
        return req.fields * self.unit


def _requests(n, seed=0, rate=200.0):
    rng = random.Random(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.expovariate(rate)
        out.append(Request(i, t, rng.choice([1, 2, 3, 5]), rng.randint(1, 20), rng.choice(["fp32", "bf16x3"])))
    return out


@pytest.mark.parametrize("slots,budget", [(1, 400), (4, 600), (8, 2000)])
def test_all_complete_within_budget_in_arrival_order(slots, budget):
    clock = MockClock()
    ex = FakeExecutor(clock)
    reqs = _requests(300, seed=slots)
    sched = Scheduler(ex, slots, budget, clock=clock, idle=clock.advance)
    done = sched.run(reqs)
    assert len(done) == len(reqs)
    assert sched.peak <= budget
    assert all(r.completed >= r.admitted >= r.arrival for r in reqs)
    # admission follows arrival order
    order = sorted(reqs, key=lambda r: (r.admitted, r.rid))
    assert [r.rid for r in order] == sorted(r.rid for r in reqs)
    assert ex.launched == sorted(ex.launched)


def test_slots_bound_concurrency():
    clock = MockClock()
    ex = FakeExecutor(clock)
    reqs = _requests(200, seed=3, rate=1e5)  # everything arrives at once
    sched = Scheduler(ex, 3, 10 ** 9, clock=clock, idle=clock.advance)
    sched.run(reqs)
    events = sorted([(r.admitted, 1) for r in reqs] + [(r.completed, -1) for r in reqs], key=lambda e: (e[0], e[1]))
    live = peak = 0
    for _t, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 3


def test_eviction_only_of_idle_tables():
    clock = MockClock()
    ex = FakeExecutor(clock, table_bytes=300)
    reqs = _requests(120, seed=7, rate=50.0)
    sched = Scheduler(ex, 2, 700, clock=clock, idle=clock.advance)
    sched.run(reqs)
    assert ex.evicted, "a 700-byte budget cannot hold every table set"
    assert sched.peak <= 700


@pytest.mark.parametrize("bypass", [1, 4])
def test_bounded_bypass_of_a_waiting_head(bypass):
    # mixed sizes under a tight budget: requests may pass a head that waits
    # for memory, at most `bypass` per waiting head; all complete in budget
    clock = MockClock()
    ex = FakeExecutor(clock, table_bytes=50)
    rng = random.Random(11)
    reqs, t = [], 0.0
    for i in range(200):
        t += rng.expovariate(400.0)
        reqs.append(Request(i, t, rng.choice([1, 2, 3]), rng.choice([1, 2, 40]), "fp32"))
    sched = Scheduler(ex, 4, 700, clock=clock, idle=clock.advance, bypass=bypass)
    done = sched.run(reqs)
    assert len(done) == len(reqs)
    assert sched.peak <= 700
    idx = {rid: k for k, rid in enumerate(ex.launched)}  # launch order
    passed_any = False
    for r in reqs:
        # r is the head of the queue once every earlier request has started;
        # count the later requests that started between then and r's start
        head_from = max([idx[q.rid] for q in reqs if q.rid < r.rid], default=-1)
        ahead = [q for q in reqs if q.rid > r.rid and head_from < idx[q.rid] < idx[r.rid]]
        assert len(ahead) <= bypass, (r.rid, len(ahead))
        passed_any |= any(idx[q.rid] < idx[r.rid] for q in reqs if q.rid > r.rid)
    assert passed_any, "no request started ahead of an earlier one"


def test_oversized_request_is_refused():
    clock = MockClock()
    ex = FakeExecutor(clock)
    sched = Scheduler(ex, 2, 150, clock=clock, idle=clock.advance)
    with pytest.raises(MemoryError):
        sched.run([Request(0, 0.0, 1, 50, "fp32")])


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0
