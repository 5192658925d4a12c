"""Serving scheduler logic on the CPU with a fake executor whose batches take
a modelled time: admission by memory budget, continuous batching, overflow
retries, rejection, cancellation, in-flight limits."""
import threading
import time
from dataclasses import dataclass

import pytest

from paper_2503_07946_amd.serve import Outcome, Request, Scheduler, run_plain


class V:
    def __init__(self, W, H):
        self.W, self.H = W, H


class FakeExecutor:
    """A batch takes `overhead + per_px * pixels` seconds after launch."""

    def __init__(self, bytes_per_px=10, overhead=0.004, per_px=2e-9, overflow_ids=()):
        self.bpp = bytes_per_px
        self.overhead = overhead
        self.per_px = per_px
        self.overflow_ids = set(overflow_ids)
        self.live_bytes = 0
        self.max_live = 0
        self.inflight = 0
        self.max_inflight = 0
        self.launched = []
        self.lock = threading.Lock()

    def footprint(self, r):
        return self.bpp * r.view.W * r.view.H

    def launch(self, reqs):
        nbytes = sum(self.footprint(r) for r in reqs)
        self.live_bytes += nbytes
        self.max_live = max(self.max_live, self.live_bytes)
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        px = sum(r.view.W * r.view.H for r in reqs)
        self.launched.append([r.rid for r in reqs])
        return (time.perf_counter() + self.overhead + self.per_px * px, list(reqs), nbytes), nbytes

    def ready(self, h):
        return time.perf_counter() >= h[0]

    def wait(self, handles, timeout):
        t = min(h[0] for h in handles) - time.perf_counter()
        if timeout is not None:
            t = min(t, timeout)
        if t > 0:
            time.sleep(t)

    def collect(self, h):
        self.live_bytes -= h[2]
        self.inflight -= 1
        out = []
        for r in h[1]:
            if r.rid in self.overflow_ids and r.attempts == 1:
                out.append(Outcome(r, False, 12345))
            else:
                out.append(Outcome(r, True, 100, result=("img", r.rid)))
        return out

    def render_one(self, r):
        time.sleep(self.overhead + self.per_px * r.view.W * r.view.H)
        return ("img", r.rid)


def _stream(n, gap, res=(64, 64)):
    return [Request(i, i * gap, i % 3, V(*res)) for i in range(n)]


def test_every_request_completes_once_within_budget():
    ex = FakeExecutor()
    budget = 10 * 64 * 64 * 5          # room for 5 frames
    reqs = _stream(60, 0.0005)
    st = Scheduler(ex, budget, max_slots=8, max_inflight=2).run(reqs)
    assert sorted(r.rid for r in st.completed) == list(range(60))
    assert all(r.status == "done" and r.result == ("img", r.rid) for r in st.completed)
    assert ex.max_live <= budget
    assert ex.max_inflight <= 2
    assert max(len(b) for b in ex.launched) <= 5
    # FIFO admission: launch order is arrival order
    flat = [i for b in ex.launched for i in b]
    assert flat == sorted(flat)


def test_continuous_batching_groups_requests_that_arrive_during_a_batch():
    ex = FakeExecutor(overhead=0.02)
    reqs = _stream(40, 0.002)
    st = Scheduler(ex, 1 << 30, max_slots=16, max_inflight=1).run(reqs)
    assert len(st.completed) == 40
    assert st.batches < 20
    assert max(st.batch_sizes) > 1


def test_two_batches_overlap_in_flight():
    ex = FakeExecutor(overhead=0.02)
    reqs = _stream(30, 0.001)
    Scheduler(ex, 1 << 30, max_slots=4, max_inflight=2).run(reqs)
    assert ex.max_inflight == 2


def test_overflow_is_retried_at_the_head_with_the_reported_size():
    ex = FakeExecutor(overflow_ids={3, 7})
    reqs = _stream(12, 0.001)
    st = Scheduler(ex, 1 << 30, max_slots=4, max_inflight=1).run(reqs)
    assert sorted(r.rid for r in st.completed) == list(range(12))
    retried = {r.rid: r for r in st.completed if r.attempts > 1}
    assert set(retried) == {3, 7}
    assert all(r.pairs_hint == 12345 for r in retried.values())
    assert st.retries == 2


class ArrayView(V):
    """A view whose == is ambiguous, as with numpy-array fields."""

    def __eq__(self, other):
        raise ValueError("ambiguous comparison")

    __hash__ = object.__hash__


@dataclass
class Handle:
    """A launch handle compared by value, its first field a view."""
    view: object
    due: float
    reqs: list
    nbytes: int


class HandleExecutor(FakeExecutor):
    def launch(self, reqs):
        (due, rs, nbytes), nb = super().launch(reqs)
        return Handle(rs[0].view, due, rs, nbytes), nb

    def ready(self, h):
        return time.perf_counter() >= h.due

    def wait(self, handles, timeout):
        t = min(h.due for h in handles) - time.perf_counter()
        if timeout is not None:
            t = min(t, timeout)
        if t > 0:
            time.sleep(t)

    def collect(self, h):
        return super().collect((h.due, h.reqs, h.nbytes))


def test_batches_completing_out_of_order_with_uncomparable_handles():
    """A later, smaller batch finishes before an earlier large one; taking it
    off the in-flight list must not compare handles or requests by value."""
    ex = HandleExecutor(overhead=0.001, per_px=2e-8)
    reqs = [Request(0, 0.0, 0, ArrayView(512, 512)), Request(1, 0.0005, 0, ArrayView(8, 8))]
    st = Scheduler(ex, 1 << 30, max_slots=1, max_inflight=2).run(reqs)
    assert sorted(r.rid for r in st.completed) == [0, 1]
    assert st.completed[0].rid == 1           # the small one finished first


def test_request_larger_than_budget_is_rejected():
    ex = FakeExecutor()
    reqs = _stream(5, 0.001)
    reqs[2] = Request(2, 0.002, 0, V(4000, 4000))
    st = Scheduler(ex, 10 * 64 * 64 * 4, max_slots=4).run(reqs)
    assert [r.rid for r in st.rejected] == [2]
    assert sorted(r.rid for r in st.completed) == [0, 1, 3, 4]


def test_queued_request_past_its_deadline_is_cancelled():
    ex = FakeExecutor(overhead=0.05)
    reqs = _stream(6, 0.0)
    for r in reqs[1:]:
        r.deadline = 0.01
    st = Scheduler(ex, 10 * 64 * 64, max_slots=1, max_inflight=1).run(reqs)
    assert [r.rid for r in st.completed] == [0]
    assert sorted(r.rid for r in st.cancelled) == [1, 2, 3, 4, 5]


def test_batched_beats_plain_under_load_in_the_model():
    """With a fixed per-launch cost, batching keeps the queue short where one
    frame per launch falls behind the arrivals."""
    reqs_a = _stream(80, 0.003)
    reqs_b = _stream(80, 0.003)
    batched = Scheduler(FakeExecutor(overhead=0.006), 1 << 30, max_slots=16, max_inflight=2).run(reqs_a)
    plain = run_plain(FakeExecutor(overhead=0.006), reqs_b)
    sb, sp = batched.summary(), plain.summary()
    assert sb["p99_ms"] < sp["p99_ms"]


def test_summary_fields():
    ex = FakeExecutor()
    st = Scheduler(ex, 1 << 30).run(_stream(10, 0.001))
    s = st.summary(skip=2)
    assert s["requests"] == 8 and s["p50_ms"] is not None and s["p99_ms"] >= s["p50_ms"]


@pytest.mark.parametrize("slots", [1, 3])
def test_slot_limit(slots):
    ex = FakeExecutor(overhead=0.01)
    Scheduler(ex, 1 << 30, max_slots=slots, max_inflight=2).run(_stream(20, 0.0))
    assert max(len(b) for b in ex.launched) <= slots
