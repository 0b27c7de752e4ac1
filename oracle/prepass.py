"""Oracle for the locality pre-pass run before Algorithm 1: the shingle ordering.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Pure Python on Python
integers, meant for small graphs.

Section 2.2 runs Gorder before JaccardWithWindows so that vertices with similar
neighbourhoods tend to fall into the same window, and does not specify Gorder
further.  The stand-in is the shingle ordering of Chierichetti, Kumar, Lattanzi,
Mitzenmacher, Panconesi and Raghavan ("On compressing social networks", KDD 2009):
each vertex is keyed by min-hashes of its out-neighbour set and vertices are sorted
by key, so that two vertices share a min-hash with probability equal to the
Jaccard similarity of their neighbour sets (the quantity Algorithm 1 maximises).

Definitions followed here
  * SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
    generators", OOPSLA 2014): the stream seeded with s has state s + t * gamma
    after t steps, gamma = 0x9E3779B97F4A7C15, and output t is the state passed
    through the 64-bit finaliser z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
    z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31 (all modulo 2^64).
  * Hash function i (i = 0 .. k-1) has seed s_i = output i + 1 of the stream
    seeded with `seed`, and h_i(u) = output u + 1 of the stream seeded with s_i.
  * key_i(v) = min over out-neighbours u of v of h_i(u); 2^64 - 1 when v has no
    out-neighbours.
  * Vertices take labels 0, 1, ... in ascending order of (key_0, ..., key_{k-1}, v).
  * The pre-pass output feeds Algorithm 1: its windows are taken over the pre-pass
    labels, and the final label of v is Algorithm 1's label of v's pre-pass label.
"""
from __future__ import annotations

import numpy as np

from . import reorder

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
EMPTY_KEY = MASK


def splitmix64(seed: int, t: int) -> int:
    """Output t (t >= 1) of the SplitMix64 stream seeded with `seed`."""
    z = (seed + t * GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def hash_table(n: int, k: int, seed: int):
    """H[i][u] = h_i(u) for i < k, u < n."""
    seeds = [splitmix64(seed, i + 1) for i in range(k)]
    return [[splitmix64(s, u + 1) for u in range(n)] for s in seeds]


def minhash_keys(g, H):
    """key[v] = (min over out-neighbours u of H[0][u], ..., of H[k-1][u])."""
    rp = g.row_ptr
    keys = []
    for v in range(g.n):
        nb = [int(u) for u in g.col[rp[v]:rp[v + 1]]]
        keys.append(tuple(min((Hi[u] for u in nb), default=EMPTY_KEY) for Hi in H))
    return keys


def shingle_order_from_hashes(g, H) -> np.ndarray:
    """new_id[v]: rank of (key(v), v) among all vertices."""
    keys = minhash_keys(g, H)
    order = sorted(range(g.n), key=lambda v: (keys[v], v))
    new_id = np.empty(g.n, dtype=np.uint32)
    for rank, v in enumerate(order):
        new_id[v] = rank
    return new_id


def shingle_order(g, k: int, seed: int) -> np.ndarray:
    return shingle_order_from_hashes(g, hash_table(g.n, k, seed))


def relabel(g, new_id):
    """The graph with vertex v renamed new_id[v] (rows sorted)."""
    class _G:
        pass
    out = _G()
    out.n = g.n
    rows = [[] for _ in range(g.n)]
    rp = g.row_ptr
    for v in range(g.n):
        rows[int(new_id[v])] = sorted(int(new_id[int(u)]) for u in g.col[rp[v]:rp[v + 1]])
    out.row_ptr = np.zeros(g.n + 1, dtype=np.uint32)
    out.row_ptr[1:] = np.cumsum([len(r) for r in rows])
    out.col = np.array([u for r in rows for u in r], dtype=np.uint32)
    return out


def prepass_then_windows(g, k: int, seed: int, sigma: int, w: int) -> np.ndarray:
    """Final label of each vertex: Algorithm 1 over the shingle-ordered graph."""
    pre = shingle_order(g, k, seed)
    win = reorder.jaccard_with_windows(relabel(g, pre), sigma, w)
    return np.asarray([win[int(pre[v])] for v in range(g.n)], dtype=np.uint32)
