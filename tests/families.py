"""Small graph families with closed-form BFS levels, built through the shared input
normaliser (``inputs.from_arcs``).  Each builder returns (graph, level_fn) where
level_fn(source) gives the exact level array from the family's closed form."""
from __future__ import annotations

import itertools

import numpy as np

import inputs


def path(n):
    g = inputs.from_arcs(n, np.arange(n - 1), np.arange(1, n), True)
    return g, lambda s: np.abs(np.arange(n) - s).astype(np.int32)


def cycle(n):
    g = inputs.from_arcs(n, np.arange(n), (np.arange(n) + 1) % n, True)

    def lv(s):
        d = np.abs(np.arange(n) - s)
        return np.minimum(d, n - d).astype(np.int32)
    return g, lv


def star(n):
    """Centre 0, leaves 1..n-1."""
    g = inputs.from_arcs(n, np.zeros(n - 1, np.int64), np.arange(1, n), True)

    def lv(s):
        out = np.full(n, 2 if s != 0 else 1, np.int32)
        out[0] = 0 if s == 0 else 1
        out[s] = 0
        return out
    return g, lv


def complete(n):
    src, dst = zip(*[(u, v) for u in range(n) for v in range(n) if u != v])
    g = inputs.from_arcs(n, src, dst, False)

    def lv(s):
        out = np.ones(n, np.int32)
        out[s] = 0
        return out
    return g, lv


def complete_bipartite(a, b):
    """Sides 0..a-1 and a..a+b-1."""
    src, dst = zip(*[(u, a + v) for u in range(a) for v in range(b)])
    g = inputs.from_arcs(a + b, src, dst, True)

    def lv(s):
        side = np.arange(a + b) < a
        out = np.where(side == (s < a), 2, 1).astype(np.int32)
        out[s] = 0
        return out
    return g, lv


def full_grid(rows, cols):
    """p = 1 grid from the shared generator: levels are Manhattan distances."""
    g = inputs.grid(rows, cols, 1.0, seed=0)

    def lv(s):
        r, c = divmod(np.arange(rows * cols), cols)
        sr, sc = divmod(s, cols)
        return (np.abs(r - sr) + np.abs(c - sc)).astype(np.int32)
    return g, lv


def hypercube(d):
    n = 1 << d
    src, dst = zip(*[(v, v ^ (1 << b)) for v in range(n) for b in range(d)])
    g = inputs.from_arcs(n, src, dst, False)

    def lv(s):
        x = np.arange(n) ^ s
        return np.array([bin(int(t)).count("1") for t in x], np.int32)
    return g, lv


def disjoint_union_paths(n1, n2):
    """Path on 0..n1-1 and path on n1..n1+n2-1 (no edge between them)."""
    s1 = list(range(n1 - 1)) + list(range(n1, n1 + n2 - 1))
    d1 = [x + 1 for x in s1]
    g = inputs.from_arcs(n1 + n2, s1, d1, True)

    def lv(s):
        idx = np.arange(n1 + n2)
        same = (idx < n1) == (s < n1)
        return np.where(same, np.abs(idx - s), -1).astype(np.int32)
    return g, lv


def isolated_plus_edge(n):
    """Vertices 0..n-1, only the edge 1-2; source 0 reaches nothing."""
    g = inputs.from_arcs(n, [1], [2], True)

    def lv(s):
        out = np.full(n, -1, np.int32)
        out[s] = 0
        if s in (1, 2):
            out[3 - s] = 1
        return out
    return g, lv


ALL_FAMILIES = {
    "path17": lambda: path(17),
    "cycle12": lambda: cycle(12),
    "cycle13": lambda: cycle(13),
    "star9": lambda: star(9),
    "complete7": lambda: complete(7),
    "k3_5": lambda: complete_bipartite(3, 5),
    "grid5x7": lambda: full_grid(5, 7),
    "hypercube5": lambda: hypercube(5),
    "union_paths": lambda: disjoint_union_paths(6, 9),
    "isolated": lambda: isolated_plus_edge(5),
}


def small_dense_csr(n, adj):
    """CSR (object with n/row_ptr/col) from a dense 0/1 matrix adj[u][v] = arc u->v,
    built with numpy only (for exhaustive enumeration)."""
    class G:
        pass
    g = G()
    g.n = n
    rows, cols = np.nonzero(adj)
    g.row_ptr = np.zeros(n + 1, np.uint32)
    np.add.at(g.row_ptr, rows + 1, 1)
    g.row_ptr = np.cumsum(g.row_ptr).astype(np.uint32)
    g.col = cols.astype(np.uint32)
    return g


def all_undirected(n):
    pairs = list(itertools.combinations(range(n), 2))
    for bits in range(1 << len(pairs)):
        adj = np.zeros((n, n), np.uint8)
        for i, (u, v) in enumerate(pairs):
            if bits >> i & 1:
                adj[u, v] = adj[v, u] = 1
        yield adj


def all_directed(n):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    for bits in range(1 << len(pairs)):
        adj = np.zeros((n, n), np.uint8)
        for i, (u, v) in enumerate(pairs):
            if bits >> i & 1:
                adj[u, v] = 1
        yield adj
