"""CPU tests of the serving loop's batch planner and trace generator."""
from __future__ import annotations

import collections

import numpy as np

from paper_2512_21967_amd.serve import Request, plan_batch, poisson_trace


def req(i, graph, k, t):
    return Request(i, graph, np.arange(k, dtype=np.uint32), t)


def fp(graph, k):
    return 1000 + 100 * k


def test_oldest_graph_first_and_packing_limit():
    pending = {"a": collections.deque([req(0, "a", 30, 2.0), req(1, "a", 30, 3.0), req(2, "a", 10, 4.0)]),
               "b": collections.deque([req(3, "b", 5, 1.0)])}
    name, take = plan_batch(pending, 10 ** 9, fp)
    assert name == "b" and [r.rid for r in take] == [3]
    pending["b"].clear()
    name, take = plan_batch(pending, 10 ** 9, fp)
    # 30 + 30 fit in 64 columns; the third (10) would make 70
    assert name == "a" and [r.rid for r in take] == [0, 1]


def test_budget_limits_the_batch_and_keeps_order():
    pending = {"a": collections.deque([req(0, "a", 10, 1.0), req(1, "a", 10, 2.0), req(2, "a", 1, 3.0)])}
    # room for 15 columns: the first request only; the later, smaller one does not jump the queue
    name, take = plan_batch(pending, fp("a", 15), fp)
    assert [r.rid for r in take] == [0]
    assert plan_batch(pending, fp("a", 5), fp) is None
    assert plan_batch({"a": collections.deque()}, 10 ** 9, fp) is None


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
