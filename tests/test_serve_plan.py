"""CPU tests of the serving loop's host side (paper_2512_21967_amd.serve): request
order, HBM-budget admission, release of finished requests, a full request ring,
the overlap count and the seeded trace generator.  A fake device server stands in
for libblest's (it finishes a request a fixed number of polls after submission)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2512_21967_amd.serve import Request, Server, overlapping_pairs, poisson_trace


class FakeGraph:
    def __init__(self, n):
        self.n = n
        self.device = 0


class FakeDevice:
    """Admits in submission order; a request is done `delay` polls after submission;
    at most `ring` unreleased requests."""

    def __init__(self, delay=3, ring=256):
        self.delay, self.ring = delay, ring
        self.next, self.polls, self.log, self.held = 0, {}, [], set()
        self.outstanding_seen = []

    def submit(self, graph, sources, out):
        if len(self.held) >= self.ring:
            return None
        t = self.next
        self.next += 1
        self.polls[t] = 0
        self.held.add(t)
        self.log.append((t, graph, len(sources), out))
        return t

    def poll(self, t):
        self.polls[t] += 1
        done = self.polls[t] >= self.delay
        return (2 if done else 1), 5, t, t + self.delay

    def release(self, t):
        assert self.polls[t] >= self.delay, "released before done"
        self.held.remove(t)


def make(budget, delay=3, ring=256, n=(100, 1000)):
    graphs = {"a": FakeGraph(n[0]), "b": FakeGraph(n[1])}
    dev = FakeDevice(delay, ring)
    srv = Server(graphs, budget, device_server=dev, alloc=lambda k, nn: ("buf", k, nn))
    return srv, dev


def trace_of(items):
    return [(0.0, g, np.arange(k, dtype=np.uint32)) for g, k in items]


def test_submission_order_is_arrival_order():
    srv, dev = make(10 ** 9)
    items = [("a", 3), ("b", 64), ("a", 1), ("b", 7)]
    reqs = srv.run(trace_of(items), realtime=False, keep=False)
    assert [(g, k) for _, g, k, _ in dev.log] == [(srv.index[g], k) for g, k in items]
    assert all(r.done_at is not None and r.released for r in reqs)
    assert srv.outstanding == 0


def test_budget_is_never_exceeded_and_head_of_line_order_kept():
    # budget: one b-request of 10 sources (40,000 bytes) at a time
    srv, dev = make(40_000, delay=5)
    items = [("b", 10), ("b", 10), ("a", 1), ("b", 5)]
    seen = []

    def on_done(r):
        seen.append(srv.outstanding)

    reqs = srv.run(trace_of(items), realtime=False, keep=False, on_done=on_done)
    assert srv.peak_bytes <= 40_000
    assert max(seen) <= 40_000
    # the small a-request did not jump ahead of the second b-request
    order = [t for t, _, _, _ in dev.log]
    assert order == sorted(order)
    assert [r.graph for r in sorted(reqs, key=lambda r: r.ticket)] == ["b", "b", "a", "b"]


def test_kept_requests_hold_their_bytes_until_released():
    srv, dev = make(40_000, delay=2)
    reqs = srv.run(trace_of([("b", 10)]), realtime=False, keep=True)
    assert srv.outstanding == 40_000 and not reqs[0].released
    srv.release(reqs[0])
    assert srv.outstanding == 0 and reqs[0].released
    with pytest.raises(RuntimeError):
        srv.run(trace_of([("b", 10), ("b", 10)]), realtime=False, keep=True)


def test_full_ring_waits_for_releases():
    srv, dev = make(10 ** 9, delay=2, ring=2)
    reqs = srv.run(trace_of([("a", 1)] * 9), realtime=False, keep=False)
    assert all(r.released for r in reqs) and len(dev.log) == 9


def test_budget_below_one_source_is_refused():
    with pytest.raises(ValueError):
        make(399)  # graph a: one source's output is 400 bytes


def test_overlapping_pairs():
    def req(a, d):
        r = Request(0, "a", np.zeros(1, np.uint32), 0.0)
        r.admit_iter, r.done_iter, r.done_at = a, d, 1.0
        return r
    assert overlapping_pairs([req(1, 5), req(5, 9)]) == 0          # back to back
    assert overlapping_pairs([req(1, 5), req(4, 9), req(2, 3)]) == 2
    assert overlapping_pairs([req(1, 100), req(2, 3), req(3, 4), req(50, 60)]) == 3


def test_poisson_trace_is_seeded_and_in_range():
    src = lambda g, seed, k: np.random.default_rng(seed).integers(0, 100, k)
    a = poisson_trace(3, 1000.0, 200, ["x", "y", "z"], src)
    b = poisson_trace(3, 1000.0, 200, ["x", "y", "z"], src)
    assert [t for t, _, _ in a] == [t for t, _, _ in b]
    ts = np.array([t for t, _, _ in a])
    assert np.all(np.diff(ts) > 0)
    assert abs(ts[-1] / 200 - 1e-3) < 3e-4            # mean gap 1 / rate
    ks = np.array([len(s) for _, _, s in a])
    assert ks.min() >= 1 and ks.max() <= 64
    assert 0.35 < np.mean(ks == 1) < 0.65
    assert {g for _, g, _ in a} == {"x", "y", "z"}
