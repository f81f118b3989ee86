"""Host logic of the serving loop (paper_2512_01027_amd/serving.py) on the
CPU: the library's batch is replaced by a stand-in that keeps the same
contract (admit -> slot or None when full; advance(k); poll -> finished
slots; take), so admission order, the fill limit, refusals and latency
bookkeeping are checked without a GPU."""
import math

import numpy as np
import pytest

from paper_2512_01027_amd import serving as SV


class FakeBatch:
    """Slots and a node budget; every resident case advances k steps per
    advance(), as the library's batch does."""

    log = []

    def __init__(self, hbm_budget, store="fp16", max_slots=64):
        self.budget, self.max_slots = hbm_budget, max_slots
        self.res = {}  # slot -> [remaining steps, nodes]
        self.next = 0
        self.refuse = 0  # answer None to this many admits first
        FakeBatch.log = []
        FakeBatch.inst = self

    def admit(self, cfg, phi, P, u, nsteps):
        if self.refuse:
            self.refuse -= 1
            return None
        nodes = cfg["nx"] * cfg["ny"] * cfg["nz"]
        used = sum(r[1] for r in self.res.values())
        if len(self.res) >= self.max_slots or used + nodes > self.budget:
            return None
        s = self.next
        self.next += 1
        self.res[s] = [nsteps, nodes]
        FakeBatch.log.append(("admit", cfg["rid"], sorted(r[1] for r in self.res.values())))
        return s

    def advance(self, k):
        for r in self.res.values():
            r[0] -= k

    def poll(self):
        return [s for s, r in self.res.items() if r[0] <= 0]

    def take(self, s):
        self.res.pop(s)

    def close(self):
        pass


def _reqs(sizes_steps):
    out = []
    for i, (n, steps) in enumerate(sizes_steps):
        cfg = {"nx": n, "ny": 1, "nz": 1, "rid": i}
        out.append(SV.Request(i, cfg, (None, None, None), steps, "droplet", 0.0, n))
    return out


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(SV.B, "Batch", FakeBatch)
    return FakeBatch


def _admitted(log):
    return [e[1] for e in log if e[0] == "admit"]


def test_fifo_admits_in_arrival_order(fake):
    reqs = _reqs([(100, 500), (10, 50), (50, 200), (5, 50), (80, 100)])
    out = SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=10 ** 9, admit_per_round=2)
    assert _admitted(fake.log) == [0, 1, 2, 3, 4]
    assert out["cases"] == 5 and out["policy"] == "fifo"
    assert all(r.done >= r.arrival for r in reqs)


def test_least_work_first_admits_smallest_work_first(fake):
    reqs = _reqs([(100, 500), (10, 50), (50, 200), (5, 50), (80, 100)])
    SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=10 ** 9, admit_per_round=1, policy="sjf")
    order = _admitted(fake.log)
    # one admission per round: the smallest remaining work (nodes x steps) next
    assert order == [3, 1, 4, 2, 0]


def test_big_fifo_runs_large_cases_one_at_a_time(fake):
    """Large requests (>= big_nodes) one at a time in arrival order; small
    ones alongside within the fill limit, passing a large one that waits."""
    reqs = _reqs([(500, 100), (600, 100), (10, 50), (20, 50), (700, 100), (30, 400)])
    SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=40, admit_per_round=8, policy="big_fifo",
                   big_nodes=400)
    log = [e for e in fake.log if e[0] == "admit"]
    order = [e[1] for e in log]
    # the first large one, then the small ones pass the waiting second large one
    assert order[:3] == [0, 2, 3]
    assert order.index(1) < order.index(4)
    for e in log:
        res = e[2]
        assert sum(1 for n in res if n >= 400) <= 1
        assert sum(n for n in res if n < 400) <= 40 or sum(1 for n in res if n < 400) == 1
    assert all(not math.isnan(r.done) for r in reqs)


def test_big_fifo_smaller_fill_beside_a_large_case(fake):
    """While a large case is resident, small ones fill up to fill_with_big
    only (one small case is always let in); with none resident, up to
    fill_nodes.  (Small cases resident before a large one arrives stay.)"""
    reqs = _reqs([(500, 100)] + [(10, 50)] * 10)
    out = SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=40, fill_with_big=15, admit_per_round=8,
                         policy="big_fifo", big_nodes=400)
    assert out["fill_with_big"] == 15
    saw_big = saw_full = False
    for e in (e for e in fake.log if e[0] == "admit"):
        res = e[2]
        small = [n for n in res if n < 400]
        if len(res) > len(small):
            saw_big = True
            assert sum(small) <= 15 or len(small) == 1
        elif sum(small) > 15:
            saw_full = True
            assert sum(small) <= 40
    assert saw_big and saw_full
    assert all(not math.isnan(r.done) for r in reqs)


def test_big_fifo_admits_a_small_request_past_the_fill_limit_after_max_wait(fake, monkeypatch):
    """Beside a large case the small-case fill is fill_with_big; a small
    request that has waited longer than max_wait is admitted past it."""
    clock = [0.0]
    monkeypatch.setattr(SV.time, "perf_counter", lambda: clock[0])
    orig_advance = FakeBatch.advance

    def advance(self, k):
        clock[0] += 1.0  # one second per advance
        orig_advance(self, k)

    monkeypatch.setattr(FakeBatch, "advance", advance)
    reqs = _reqs([(500, 1000)] + [(10, 400)] * 3)
    for r in reqs:
        r.arrival = 0.0
    SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=40, fill_with_big=10, admit_per_round=8,
                   policy="big_fifo", big_nodes=400, max_wait=2.5)
    log = [e for e in fake.log if e[0] == "admit"]
    # the large case and one small one at once; the others only once they
    # have waited past max_wait (3 advances), with the large case still running
    first = [e for e in log if e[1] in (0, 1)]
    assert len(first) == 2
    late = [e for e in log if e[1] in (2, 3)]
    assert len(late) == 2 and all(500 in e[2] for e in late)
    # past max_wait both join the first small case (without the bound they
    # would wait for it to finish, one at a time)
    assert any(e[2] == [10, 10, 10, 500] for e in late)
    assert all(not math.isnan(r.done) for r in reqs)


def test_fill_limit_and_refusals(fake):
    reqs = _reqs([(60, 100)] * 6 + [(250, 50)])
    orig_init = FakeBatch.__init__

    def init(self, *a, **kw):
        orig_init(self, *a, **kw)
        self.refuse = 3  # the library answers EAGAIN three times first

    FakeBatch.__init__ = init
    try:
        out = SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=200, admit_per_round=4)
    finally:
        FakeBatch.__init__ = orig_init
    # every request completes, in spite of the refusals
    assert out["cases"] == 7 and all(not math.isnan(r.done) for r in reqs)
    # resident nodes stay within the fill limit, except one case larger than
    # the limit admitted alone
    for e in fake.log:
        resident = e[2]
        assert sum(resident) <= 200 or len(resident) == 1


def test_poisson_arrivals_respected(fake):
    reqs = _reqs([(20, 100)] * 8)
    SV.set_arrivals(reqs, 400.0, seed=2)  # mean gap 2.5 ms
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr) and arr[0] > 0
    out = SV.run_batched(reqs, hbm_budget=10 ** 9, k=50, fill_nodes=10 ** 9)
    assert all(r.done >= r.arrival for r in reqs)
    assert out["latency_p99_s"] >= out["latency_p50_s"] >= 0
    # a burst puts every arrival at 0
    SV.set_arrivals(reqs, None)
    assert all(r.arrival == 0.0 and math.isnan(r.done) for r in reqs)


def test_unknown_policy_rejected(fake):
    with pytest.raises(ValueError):
        SV.run_batched(_reqs([(10, 10)]), hbm_budget=10 ** 9, policy="lifo")


def test_stream_is_seeded():
    a = SV.make_stream(6, "fp16", 0.1, case_seed=3, max_nodes=48 ** 3)
    b = SV.make_stream(6, "fp16", 0.1, case_seed=3, max_nodes=48 ** 3)
    assert [(r.cfg["nx"], r.cfg["ny"], r.cfg["nz"], r.steps, r.kind) for r in a] == \
           [(r.cfg["nx"], r.cfg["ny"], r.cfg["nz"], r.steps, r.kind) for r in b]
    for r, s in zip(a, b):
        assert np.array_equal(r.fields[0], s.fields[0])
        assert r.nodes == r.cfg["nx"] * r.cfg["ny"] * r.cfg["nz"] <= 48 ** 3
