"""Admission logic of the request loop (host only): arrival order for memory,
oversized requests served alone, one request at a time per stripe in arrival
order, requests whose graph is still being built passed over, tick size."""

import pytest


class FakeEntry:
    def __init__(self, ready=True):
        self._ready = ready

    def ready(self):
        return self._ready


def make(kind, fp, stripe=None, ready=True, rid=None):
    from paper_1702_07409_amd.serve import Request
    r = Request(kind, stripe=stripe, rid=rid)
    r.entry = FakeEntry(ready)
    r.fp = fp
    return r


def sched(budget=100, max_items=64):
    from paper_1702_07409_amd.serve import Scheduler
    return Scheduler(budget, max_items, lambda r: r.fp)


def ids(batch):
    return [r.rid for r in batch]


def test_arrival_order_for_memory():
    s = sched(100)
    for rid, fp in (("a", 60), ("b", 60), ("c", 10)):
        s.submit(make("encode", fp, rid=rid))
    # something is in flight: b does not fit, and c may not pass it
    assert ids(s.admit(inflight=1)) == ["a"]
    assert s.used == 60
    assert ids(s.admit(inflight=1)) == []
    a_done = make("encode", 60)
    a_done.footprint = 60
    s.release(a_done)
    assert ids(s.admit(inflight=0)) == ["b", "c"]
    assert s.used == 70


def test_request_above_the_budget_runs_alone():
    s = sched(100)
    s.submit(make("encode", 500, rid="big"))
    s.submit(make("encode", 5, rid="small"))
    assert ids(s.admit(inflight=1)) == []          # waits for the device to drain
    assert ids(s.admit(inflight=0)) == ["big"]     # then runs by itself
    assert ids(s.admit(inflight=1)) == []


def test_one_request_per_stripe_in_arrival_order():
    s = sched(1000)
    r1 = make("decode", 10, stripe=5, rid=1)
    r2 = make("update", 10, stripe=5, rid=2)
    r3 = make("repair", 10, stripe=7, rid=3)
    r4 = make("decode", 10, stripe=5, rid=4)
    for r in (r1, r2, r3, r4):
        s.submit(r)
    assert ids(s.admit(inflight=0)) == [1, 3]
    assert ids(s.admit(inflight=1)) == []          # stripe 5 is held by request 1
    s.release(r1)
    assert ids(s.admit(inflight=1)) == [2]         # request 2 before request 4
    s.release(r3)
    s.release(r2)
    assert ids(s.admit(inflight=0)) == [4]
    s.release(r4)
    assert s.used == 0 and not s.busy


def test_requests_with_graphs_in_build_are_passed_over():
    s = sched(1000)
    slow = make("encode", 10, ready=False, rid="slow")
    fast = make("encode", 10, rid="fast")
    s.submit(slow)
    s.submit(fast)
    assert ids(s.admit(inflight=0)) == ["fast"]
    slow.entry._ready = True
    assert ids(s.admit(inflight=1)) == ["slow"]


def test_tick_size_is_capped():
    s = sched(10 ** 9, max_items=3)
    for i in range(7):
        s.submit(make("encode", 1, rid=i))
    assert ids(s.admit(inflight=0)) == [0, 1, 2]
    assert ids(s.admit(inflight=1)) == [3, 4, 5]
    assert ids(s.admit(inflight=2)) == [6]
