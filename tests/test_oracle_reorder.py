"""Pins for the ordering oracle (``oracle.reorder``): hand-worked runs of Algorithm 1
(JaccardWithWindows) that exercise pop order, the tie rule and the growth of U;
permutation and window properties; the social-like test (Section 2.2.1) on graphs
whose class is obvious; and bandwidth closed forms for reverse Cuthill-McKee."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

import inputs
from oracle import reorder
from tests import families


def directed(n, adjacency: dict):
    src = [u for u, vs in adjacency.items() for _ in vs]
    dst = [v for vs in adjacency.values() for v in vs]
    return inputs.from_arcs(n, src, dst, False)


def test_alg1_twin_groups():
    # window 0 = 0..7: evens share {8, 9}, odds share {10, 11}; window 1 has no arcs
    adj = {v: ([8, 9] if v % 2 == 0 else [10, 11]) for v in range(8)}
    g = directed(16, adj)
    new_id = reorder.jaccard_with_windows(g, sigma=4, w=8)
    assert new_id.tolist() == [0, 4, 1, 5, 2, 6, 3, 7] + list(range(8, 16))


def test_alg1_ties_go_to_smallest_id():
    # from seed 0 (U = {4, 5}), candidates 2 and 3 both score 1/2: 2 goes first
    g = directed(8, {0: [4, 5], 1: [6], 2: [4], 3: [5]})
    new_id = reorder.jaccard_with_windows(g, sigma=4, w=4)
    assert new_id.tolist()[:4] == [0, 3, 1, 2]


def test_alg1_union_grows():
    # U = {4} picks 2 (J = 1/3 beats 1/4); then U = {4, 5, 6} makes 1 (J = 2/3) beat 3
    g = directed(12, {0: [4], 1: [5, 6], 2: [4, 5, 6], 3: [4, 8, 9, 10]})
    new_id = reorder.jaccard_with_windows(g, sigma=4, w=4)
    assert new_id.tolist()[:4] == [0, 2, 1, 3]


def test_alg1_empty_neighbourhoods_keep_order():
    g = directed(20, {})
    assert reorder.jaccard_with_windows(g, sigma=4, w=8).tolist() == list(range(20))


@pytest.mark.parametrize("w,sigma", [(8, 4), (16, 8), (24, 8)])
def test_alg1_permutation_within_windows(w, sigma):
    g = inputs.rmat_workload(8, 8, seed=2, permute_seed=3)
    new_id = reorder.jaccard_with_windows(g, sigma=sigma, w=w)
    assert sorted(new_id.tolist()) == list(range(g.n))
    win = np.arange(g.n) // w
    assert np.all(new_id // w == win)
    # each cluster start is the smallest remaining vertex of the window
    for s_k in range(0, g.n, w):
        seeds = [int(np.flatnonzero(new_id == p)[0]) for p in range(s_k, min(g.n, s_k + w), sigma)]
        assert seeds == sorted(seeds)


def test_social_like_classes():
    assert reorder.is_social_like(families.star(200)[0])
    assert not reorder.is_social_like(families.path(200)[0])
    assert not reorder.is_social_like(inputs.grid(64, 64, 0.9, seed=1))
    assert reorder.is_social_like(inputs.rmat(14, 16, seed=1))
    assert not reorder.is_social_like(directed(10, {}))


def test_power_law_fit_exact_line():
    # counts c(d) = 2^12 * d^-2 for d = 1, 2, 4, 8, 16, 32: slope -2, R^2 = 1
    deg = np.concatenate([np.full(int(4096 / d ** 2), d) for d in (1, 2, 4, 8, 16, 32, 64)])
    slope, r2, ok = reorder.power_law_fit(deg)
    assert slope == pytest.approx(-2.0) and r2 == pytest.approx(1.0) and ok


def scipy_rcm_bandwidth(g):
    m = sp.csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    order = reverse_cuthill_mckee(m, symmetric_mode=True)
    new = np.empty(g.n, np.int64)
    new[order] = np.arange(g.n)
    return reorder.bandwidth(g, new)


def test_rcm_path_and_cycle():
    g, _ = families.path(50)
    h = inputs.relabel(g, inputs.permutation(50, 4))
    assert reorder.bandwidth(h) > 1
    assert reorder.bandwidth(h, reorder.rcm(h)) == 1
    g, _ = families.cycle(50)
    h = inputs.relabel(g, inputs.permutation(50, 4))
    assert reorder.bandwidth(h, reorder.rcm(h)) == 2


@pytest.mark.parametrize("rows,cols", [(5, 7), (8, 8), (6, 20), (12, 9)])
def test_rcm_full_grid_bandwidth(rows, cols):
    g = inputs.grid(rows, cols, 1.0, seed=0)
    h = inputs.relabel(g, inputs.permutation(g.n, 3))
    new_id = reorder.rcm(h)
    assert sorted(new_id.tolist()) == list(range(h.n))
    bw = reorder.bandwidth(h, new_id)
    assert bw <= min(rows, cols) + 1
    assert bw <= scipy_rcm_bandwidth(h) + 1


def test_rcm_components_are_contiguous():
    g, _ = families.disjoint_union_paths(7, 11)
    h = inputs.relabel(g, inputs.permutation(g.n, 8))
    new_id = reorder.rcm(h)
    from scipy.sparse.csgraph import connected_components
    m = sp.csr_matrix((np.ones(h.nnz), h.col.astype(np.int64), h.row_ptr.astype(np.int64)), shape=(h.n, h.n))
    _, lab = connected_components(m, directed=False)
    for c in np.unique(lab):
        ids = np.sort(new_id[lab == c])
        assert ids[-1] - ids[0] == len(ids) - 1
