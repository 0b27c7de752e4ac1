"""Oracle for the multi-source analytics built on the k-source BFS.

TEST INFRASTRUCTURE ONLY (see the package docstring): only ``tests/``, the smoke
check and the benchmark's CPU leg may use it.

Section 2 of the paper notes that stacking k frontiers as the columns of one
bit-matrix serves multi-source problems such as centrality and diameter
computations.  These functions state those quantities by their definitions over
the level arrays of the plain FIFO BFS (``oracle.bfs_multi``):

  * per source s: reached r(s) = |{v : d(s, v) finite}|, total T(s) = sum of the
    finite d(s, v), eccentricity e(s) = max finite d(s, v), and the farthest
    vertex = the smallest vertex ID at distance e(s);
  * closeness C(s) = (r(s) - 1) / T(s) (the reciprocal of the mean distance to the
    other reached vertices; 0 when s reaches nothing else);
  * diameter bounds by iterated sweeps: every BFS gives e(s) <= D, where D is the
    largest finite distance in the graph; the next sweep starts from the farthest
    vertices of the last one.  On a connected undirected graph D <= 2 e(s) for any
    s, by the triangle inequality through s.
"""
from __future__ import annotations

import numpy as np

from . import bfs_multi


def source_stats(levels: np.ndarray) -> dict:
    """levels: int32 [k, n] (or [n]); -1 = unreached.  Returns per-row arrays."""
    lv = np.atleast_2d(np.asarray(levels, dtype=np.int64))
    k, n = lv.shape
    reached = np.zeros(k, np.uint64)
    total = np.zeros(k, np.uint64)
    ecc = np.full(k, -1, np.int32)
    far = np.full(k, 0xFFFFFFFF, np.uint32)
    close = np.zeros(k, np.float64)
    for j in range(k):
        fin = lv[j] >= 0
        reached[j] = int(fin.sum())
        total[j] = int(lv[j][fin].sum())
        if reached[j]:
            ecc[j] = int(lv[j][fin].max())
            far[j] = int(np.flatnonzero(lv[j] == ecc[j])[0])
        close[j] = (float(reached[j]) - 1.0) / float(total[j]) if total[j] else 0.0
    return {"reached": reached, "total": total, "ecc": ecc, "far": far, "closeness": close}


def closeness(g, sources) -> np.ndarray:
    return source_stats(bfs_multi(g, sources))["closeness"]


def diameter_bounds(g, sources, sweeps: int = 2, undirected: bool = True):
    """(lower, upper, sweep_sources): lower = the largest eccentricity seen over
    `sweeps` rounds, each round a BFS from every current source, the next round's
    sources being the distinct farthest vertices of this one (at most 64 per round,
    in first-seen order).  upper = 2 * min e(s) over rows that reached all n
    vertices (the graph is then connected), if the graph is undirected; else None."""
    src = [int(s) for s in sources][:64]
    lower, upper, used = -1, None, []
    for _ in range(max(1, sweeps)):
        st = source_stats(bfs_multi(g, src))
        used.append(list(src))
        lower = max(lower, int(st["ecc"].max()))
        for j in range(len(src)):
            if undirected and int(st["reached"][j]) == g.n:
                u = 2 * int(st["ecc"][j])
                upper = u if upper is None else min(upper, u)
        nxt = []
        for f in st["far"]:
            f = int(f)
            if f != 0xFFFFFFFF and f not in nxt:
                nxt.append(f)
        src = nxt[:64]
    return lower, upper, used
