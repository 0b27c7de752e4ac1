"""Oracle for the host-side orderings: JaccardWithWindows (Algorithm 1), the
social-like test (Section 2.2.1) and reverse Cuthill-McKee.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Pure Python, meant for small
graphs: every argmax scans the whole remaining window.

Readings of points the paper leaves open
  * N(j) is column j of A in CSC, i.e. the out-neighbours of j in G (A is the
    adjacency of the transposed graph).
  * pop(Q) returns the smallest remaining vertex ID of the window; the argmax breaks
    ties towards the smallest vertex ID; the Jaccard similarity of two empty sets is 0.
  * Windows are [k*w, min(n, (k+1)*w)) in the input labels (no pre-pass).
  * The output maps each vertex to its new ID (the paper's pi^{-1}).
  * Social-like (Section 2.2.1): heavy tail = the ceil(1%) highest-degree vertices
    hold more than 5% of the degree sum AND the ceil(10%) highest hold more than 40%;
    power law = a least-squares line through (log d, log count(d)) over degrees
    d >= 1 with count > 0 (at least 3 such degrees) has slope in [-3.5, -1.5] and
    R^2 >= 0.9.  Social-like iff either holds.
  * RCM works on the undirected view (out- plus in-neighbours), which is the graph
    itself for the symmetric inputs used here.  Components in order of their smallest vertex ID; each starts at a
    George-Liu pseudo-peripheral vertex found from the component's minimum-degree
    vertex (ties: smallest ID), moving to the minimum-degree vertex of the last BFS
    level while the eccentricity grows; Cuthill-McKee visits the unvisited
    neighbours of each dequeued vertex in (degree, ID) order; the concatenated order
    is reversed at the end.
"""
from __future__ import annotations

import math

import numpy as np


def _neighbours(g):
    rp = g.row_ptr
    return [set(int(x) for x in g.col[rp[v]:rp[v + 1]]) for v in range(g.n)]


def _undirected_neighbours(g):
    """N(v) = out(v) | in(v); RCM orders the undirected view of the graph."""
    N = _neighbours(g)
    for v in range(g.n):
        for w in list(N[v]):
            N[w].add(v)
    return N


def _jaccard(a: set, b: set) -> float:
    union = len(a | b)
    return 0.0 if union == 0 else len(a & b) / union


def jaccard_with_windows(g, sigma: int, w: int) -> np.ndarray:
    """Algorithm 1.  Returns new_id[old] (uint32[n])."""
    assert w % sigma == 0 and w > 0
    N = _neighbours(g)
    new_id = np.full(g.n, -1, dtype=np.int64)
    for s_k in range(0, g.n, w):
        e_k = min(g.n, s_k + w)
        Q = list(range(s_k, e_k))                # kept ascending
        L_k = e_k - s_k
        M_k = -(-L_k // sigma)
        for ell in range(M_k):
            j_star = Q.pop(0)                      # pop: smallest remaining ID
            new_id[j_star] = s_k + ell * sigma
            U = set(N[j_star])
            for r in range(1, sigma):
                if not Q:
                    break
                best, best_j = -1.0, None
                for j in Q:                         # ascending: first max wins ties
                    sim = _jaccard(N[j], U)
                    if sim > best:
                        best, best_j = sim, j
                Q.remove(best_j)
                new_id[best_j] = s_k + ell * sigma + r
                U |= N[best_j]
    assert (new_id >= 0).all()
    return new_id.astype(np.uint32)


def is_social_like(g) -> bool:
    deg = np.diff(g.row_ptr.astype(np.int64))
    total = int(deg.sum())
    if total == 0:
        return False
    d_sorted = np.sort(deg)[::-1]
    top1 = max(1, math.ceil(0.01 * g.n))
    top10 = max(1, math.ceil(0.10 * g.n))
    heavy = d_sorted[:top1].sum() / total > 0.05 and d_sorted[:top10].sum() / total > 0.40
    return bool(heavy or power_law_fit(deg)[2])


def power_law_fit(deg):
    """(slope, r2, accepted) of the log-log degree-histogram line."""
    d = deg[deg >= 1]
    if d.size == 0:
        return 0.0, 0.0, False
    vals, counts = np.unique(d, return_counts=True)
    if vals.size < 3:
        return 0.0, 0.0, False
    x = np.log(vals.astype(np.float64))
    y = np.log(counts.astype(np.float64))
    xm, ym = x.mean(), y.mean()
    sxx = ((x - xm) ** 2).sum()
    sxy = ((x - xm) * (y - ym)).sum()
    slope = sxy / sxx
    resid = y - (ym + slope * (x - xm))
    syy = ((y - ym) ** 2).sum()
    r2 = 1.0 - (resid ** 2).sum() / syy if syy > 0 else 0.0
    return float(slope), float(r2), bool(-3.5 <= slope <= -1.5 and r2 >= 0.9)


def _eccentricity(N, root):
    """(eccentricity of root, vertices of its last BFS level)."""
    level = {root: 0}
    frontier = [root]
    last = [root]
    while frontier:
        nxt = []
        for v in frontier:
            for w in sorted(N[v]):
                if w not in level:
                    level[w] = level[v] + 1
                    nxt.append(w)
        if nxt:
            last = nxt
        frontier = nxt
    ecc = max(level.values())
    return ecc, last


def rcm(g) -> np.ndarray:
    """Reverse Cuthill-McKee on the undirected view.  Returns new_id[old] (uint32[n])."""
    N = [sorted(s) for s in _undirected_neighbours(g)]
    deg = [len(x) for x in N]
    seen = [False] * g.n
    order = []
    for start in range(g.n):
        if seen[start]:
            continue
        # the component of `start` (its smallest vertex ID, scanning upwards)
        comp = []
        stack = [start]
        inside = {start}
        while stack:
            v = stack.pop()
            comp.append(v)
            for w in N[v]:
                if w not in inside:
                    inside.add(w)
                    stack.append(w)
        x = min(comp, key=lambda v: (deg[v], v))
        ecc, last = _eccentricity(N, x)
        while True:
            y = min(last, key=lambda v: (deg[v], v))
            ecc_y, last_y = _eccentricity(N, y)
            if ecc_y > ecc:
                x, ecc, last = y, ecc_y, last_y
            else:
                break
        # Cuthill-McKee from x
        seen[x] = True
        queue = [x]
        head = 0
        while head < len(queue):
            v = queue[head]
            head += 1
            for w in sorted((w for w in N[v] if not seen[w]), key=lambda u: (deg[u], u)):
                seen[w] = True
                queue.append(w)
        order.extend(queue)
    order.reverse()
    new_id = np.empty(g.n, dtype=np.uint32)
    new_id[np.array(order, dtype=np.int64)] = np.arange(g.n, dtype=np.uint32)
    return new_id


def bandwidth(g, new_id=None) -> int:
    """max |new_id[u] - new_id[v]| over arcs (identity labels if new_id is None)."""
    deg = np.diff(g.row_ptr.astype(np.int64))
    u = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    v = g.col.astype(np.int64)
    if new_id is not None:
        u = new_id.astype(np.int64)[u]
        v = new_id.astype(np.int64)[v]
    return int(np.abs(u - v).max()) if u.size else 0
