"""Runs the oracle's single-source BFS for many (graph, source) pairs on host
threads.  The oracle itself is unchanged and single-threaded; the C call releases
the interpreter lock, so independent sources run in parallel."""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

import oracle

# the GPU machine grants 16 host threads per GPU
THREADS = max(1, min(16, os.cpu_count() or 1))


def rows(gr, sources, threads: int = THREADS) -> np.ndarray:
    """int32[k, n]: row j is the oracle's BFS of `gr` from sources[j]."""
    src = [int(s) for s in sources]
    out = np.empty((len(src), gr.n), dtype=np.int32)
    oracle.bfs(gr, src[0]) if src else None  # loads the library once, outside the pool
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        for j, lv in enumerate(ex.map(lambda s: oracle.bfs(gr, s), src)):
            out[j] = lv
    return out


def each(pairs, threads: int = THREADS):
    """Levels of oracle.bfs(g, s) for every (g, s) in `pairs`, in order."""
    pairs = list(pairs)
    if not pairs:
        return []
    oracle.bfs(pairs[0][0], int(pairs[0][1]))
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda p: oracle.bfs(p[0], int(p[1])), pairs))
