"""Pins of the shingle pre-pass oracle (the stand-in for Gorder before Algorithm 1,
Section 2.2): the hash generator against published test vectors, the min-hash key
and the sort on a hand-worked case, the min-hash collision probability against the
Jaccard similarity, and the composition with Algorithm 1 on planted twin groups,
where the optimal slice count is known in closed form."""
from __future__ import annotations

import os

import numpy as np
import pytest

import inputs
from oracle import bvss as obvss
from oracle import prepass
from oracle import reorder as oreorder

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64.txt")) if not l.startswith("#")]
    assert len(rows) == 8
    for seed, t, out in rows:
        assert prepass.splitmix64(int(seed), int(t)) == int(out)


def _graph(n, adj):
    src = [u for u, vs in adj.items() for _ in vs]
    dst = [v for vs in adj.values() for v in vs]
    return inputs.from_arcs(n, src, dst, False)


def test_hand_worked_order():
    # out-neighbours: 0 -> {1, 2}, 1 -> {3}, 2 -> {1, 4}, 3 -> {}, 4 -> {0, 5}, 5 -> {2, 3}
    g = _graph(6, {0: [1, 2], 1: [3], 2: [1, 4], 4: [0, 5], 5: [2, 3]})
    h0 = [50, 10, 40, 30, 20, 60]
    # keys 10, 30, 10, empty, 50, 30 -> order 0, 2, 1, 5, 4, 3 (ties by ID)
    assert prepass.minhash_keys(g, [h0]) == [(10,), (30,), (10,), (prepass.EMPTY_KEY,), (50,), (30,)]
    np.testing.assert_array_equal(prepass.shingle_order_from_hashes(g, [h0]), [0, 2, 1, 5, 4, 3])
    # a second hash breaks the ties: v2 (min(8, 1) = 1) before v0 (min(8, 3) = 3),
    # v5 (min(3, 6) = 3) before v1 (6) -> order 2, 0, 5, 1, 4, 3
    h1 = [5, 8, 3, 6, 1, 4]
    np.testing.assert_array_equal(prepass.shingle_order_from_hashes(g, [h0, h1]), [1, 3, 0, 5, 4, 2])


def test_collision_probability_is_the_jaccard_similarity():
    # N(0) = {2, 3, 4, 5}, N(1) = {4, 5, 6}: Jaccard 2 / 5
    g = _graph(7, {0: [2, 3, 4, 5], 1: [4, 5, 6]})
    trials = 3000
    same = 0
    for seed in range(trials):
        k0, k1 = prepass.minhash_keys(g, prepass.hash_table(7, 1, seed))[:2]
        same += k0 == k1
    sd = (0.4 * 0.6 / trials) ** 0.5
    assert abs(same / trials - 0.4) < 5 * sd


def test_keys_are_neighbourhood_minima_by_brute_force():
    rng = np.random.default_rng(3)
    n = 40
    gr = inputs.from_arcs(n, rng.integers(0, n, 120), rng.integers(0, n, 120), False)
    H = prepass.hash_table(n, 3, 99)
    keys = prepass.minhash_keys(gr, H)
    for v in range(n):
        nb = set(int(u) for u in gr.col[gr.row_ptr[v]:gr.row_ptr[v + 1]])
        for i in range(3):
            want = prepass.EMPTY_KEY if not nb else sorted(H[i][u] for u in nb)[0]
            assert keys[v][i] == want
    new_id = prepass.shingle_order_from_hashes(gr, H)
    assert sorted(new_id.tolist()) == list(range(n))
    # ascending keys along the new labels
    by_label = [None] * n
    for v in range(n):
        by_label[new_id[v]] = (keys[v], v)
    assert by_label == sorted(by_label)


def _planted_twins(groups, sigma, fan, seed):
    """groups * sigma vertices in twin groups of sigma (identical out-neighbour
    sets, disjoint between groups, each of `fan` target vertices that have no
    out-arcs), labels shuffled."""
    rng = np.random.default_rng(seed)
    n = groups * sigma + groups * fan
    src, dst = [], []
    for gi in range(groups):
        targets = groups * sigma + gi * fan + np.arange(fan)
        for j in range(sigma):
            for t in targets:
                src.append(gi * sigma + j)
                dst.append(int(t))
    g = inputs.from_arcs(n, src, dst, False)
    return inputs.relabel(g, inputs.permutation(n, seed)), n


def _num_slices(g, new_id, sigma):
    h = prepass.relabel(g, new_id)
    return obvss.slices(h, sigma)[0].size


@pytest.mark.parametrize("sigma", [8, 16])
def test_prepass_then_windows_recovers_planted_twin_groups(sigma):
    groups, fan = 6, 5
    g, n = _planted_twins(groups, sigma, fan, seed=sigma)
    # each twin group in one slice set gives fan slices per group: the minimum
    # (every arc needs a slice, and a slice holds at most sigma arcs, here all twins)
    optimum = groups * fan
    # windows of one slice set cannot bring scattered twins together ...
    alone = oreorder.jaccard_with_windows(g, sigma, sigma)
    assert _num_slices(g, alone, sigma) > optimum
    # ... the pre-pass makes each group contiguous and sigma-aligned first
    both = prepass.prepass_then_windows(g, 2, 0x243F6A8885A308D3, sigma, sigma)
    assert sorted(both.tolist()) == list(range(n))
    assert _num_slices(g, both, sigma) == optimum
