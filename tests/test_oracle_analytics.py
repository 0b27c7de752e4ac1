"""Pins for the multi-source analytics oracle (``oracle.analytics``): closed forms
on families whose distances are known, scipy's all-pairs shortest paths on random
graphs (an independent BFS), and the sweep bounds on graphs whose diameter is known.
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import inputs
from oracle import analytics
from tests import families


def _one(g, s):
    st = analytics.source_stats(analytics.bfs_multi(g, [s]))
    return {k: v[0] for k, v in st.items()}


def test_path_end_and_middle():
    n = 17
    g, _ = families.path(n)
    a = _one(g, 0)
    assert (a["reached"], a["total"], a["ecc"], a["far"]) == (n, n * (n - 1) // 2, n - 1, n - 1)
    assert a["closeness"] == pytest.approx(2.0 / n, rel=0, abs=1e-15)
    m = (n - 1) // 2
    b = _one(g, m)
    # both ends are at distance m; the smaller ID is reported
    assert (b["total"], b["ecc"], b["far"]) == (m * (m + 1), m, 0)


def test_star_centre_and_leaf():
    n = 9
    g, _ = families.star(n)
    c = _one(g, 0)
    assert (c["total"], c["ecc"], c["far"], c["closeness"]) == (n - 1, 1, 1, 1.0)
    for s, far in ((1, 2), (4, 1)):
        leaf = _one(g, s)
        assert (leaf["total"], leaf["ecc"], leaf["far"]) == (1 + 2 * (n - 2), 2, far)
        assert leaf["closeness"] == (n - 1) / (2 * n - 3)


@pytest.mark.parametrize("n", [12, 13])
def test_cycle(n):
    g, _ = families.cycle(n)
    m = n // 2
    for s in (0, 5):
        a = _one(g, s)
        assert a["ecc"] == m
        assert a["total"] == (m * m if n % 2 == 0 else m * (m + 1))
        assert a["far"] == (min((s + m) % n, (s - m) % n))


def test_full_grid_corner():
    r, c = 5, 7
    g, _ = families.full_grid(r, c)
    a = _one(g, 0)
    assert (a["ecc"], a["far"]) == (r + c - 2, r * c - 1)
    assert a["total"] == c * r * (r - 1) // 2 + r * c * (c - 1) // 2


def test_unreached_and_isolated():
    g, _ = families.disjoint_union_paths(6, 9)
    a = _one(g, 2)
    assert (a["reached"], a["ecc"], a["total"]) == (6, 3, 2 + 1 + 0 + 1 + 2 + 3)
    g, _ = families.isolated_plus_edge(5)
    b = _one(g, 0)
    assert (b["reached"], b["total"], b["ecc"], b["far"], b["closeness"]) == (1, 0, 0, 0, 0.0)


def test_against_all_pairs_shortest_paths():
    rng = np.random.default_rng(7)
    for trial in range(4):
        n = 40 + 10 * trial
        m = 2 * n
        g = inputs.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), trial % 2 == 0)
        A = sp.csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(n, n))
        D = shortest_path(A, method="D", directed=True, unweighted=True)
        srcs = list(range(0, n, 3))
        st = analytics.source_stats(analytics.bfs_multi(g, srcs))
        for j, s in enumerate(srcs):
            fin = np.isfinite(D[s])
            d = D[s][fin].astype(np.int64)
            assert st["reached"][j] == fin.sum()
            assert st["total"][j] == d.sum()
            assert st["ecc"][j] == d.max()
            assert st["far"][j] == np.flatnonzero(fin & (D[s] == d.max()))[0]
            want = (fin.sum() - 1) / d.sum() if d.sum() else 0.0
            assert st["closeness"][j] == want


def test_diameter_bounds_known_diameters():
    # path: the second sweep from an end reaches the other end, and 2 e(middle) = n - 1
    g, _ = families.path(17)
    lo, up, used = analytics.diameter_bounds(g, [8], sweeps=2)
    assert (lo, up) == (16, 16) and used == [[8], [0]]
    # grid: any start reaches a corner within two sweeps
    g, _ = families.full_grid(5, 7)
    lo, up, _ = analytics.diameter_bounds(g, [17], sweeps=3)
    assert lo == 10 and up >= 10
    # hypercube: every vertex has eccentricity d
    g, _ = families.hypercube(5)
    assert analytics.diameter_bounds(g, [0, 9], sweeps=2)[:2] == (5, 10)
    # disconnected: no upper bound from a row that misses vertices
    g, _ = families.disjoint_union_paths(6, 9)
    lo, up, _ = analytics.diameter_bounds(g, [0, 6], sweeps=2)
    assert (lo, up) == (8, None)
