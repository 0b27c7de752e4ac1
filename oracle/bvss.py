"""Oracle for the Binarised Virtual Slice Set (BVSS) structure and its statistics.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy/Python written
from the definitions in the paper; no blocking or layout tricks.

Definitions followed
  * Slices (Section 2): A is the adjacency of the transposed graph, so row u of A
    lists the in-neighbours of u.  Columns are cut into intervals of sigma; the slice
    of row u in interval i exists iff u has an in-neighbour in [sigma*i, sigma*i+sigma),
    and bit j of its mask is A[u][sigma*i + j], i.e. set iff the arc
    (sigma*i + j) -> u exists.  Bit 0 is the lowest column (least significant bit).
  * Virtual slice sets (Section 2.1, rules 1 and 2): every VSS holds at most tau
    slices, all from one slice set; a slice set without slices has no VSS.  The
    slices of a set are sorted by row ID (Section 2.1.2) and cut into consecutive
    groups of tau, so only the last VSS of a set can be short.  ``realPtrs[s]`` ..
    ``realPtrs[s+1]`` is the VSS range of set s and ``virtualToReal[v]`` the set of
    VSS v (Section 2.1).
  * Column-major placement (Section 2.1.2): the k-th slice of a VSS (in row order)
    goes to lane k mod lanes, slot floor(k / lanes).
  * Compression ratio (Section 2.2): m / (numSlices * sigma) over unpadded slices.
  * Update divergence (Section 2.2.1): for each slot column of the lanes x slots
    distribution matrix, the population standard deviation of the row IDs of the
    (unpadded) slices in it; a VSS's divergence is the mean over its non-empty
    columns; the graph's is the mean over all VSSs.
  * Table 3 byte accounting: a stored slice costs a 4-byte row ID plus a sigma-bit
    mask, and realPtrs and virtualToReal cost 4 bytes per entry.
"""
from __future__ import annotations

import numpy as np


def slices(g, sigma: int):
    """All slices of the transposed adjacency, sorted by (slice set, row).

    Returns (set_id int64[S], row int64[S], mask uint64[S])."""
    deg = np.diff(g.row_ptr.astype(np.int64))
    tail = np.repeat(np.arange(g.n, dtype=np.int64), deg)      # v in arc v -> u
    head = g.col.astype(np.int64)                              # u (the pulling row)
    set_of_arc = tail // sigma
    bit_of_arc = np.left_shift(np.uint64(1), (tail % sigma).astype(np.uint64))
    key = set_of_arc * g.n + head
    order = np.argsort(key, kind="stable")
    key = key[order]
    bits = bit_of_arc[order]
    if key.size == 0:
        e = np.zeros(0, np.int64)
        return e, e, np.zeros(0, np.uint64)
    starts = np.flatnonzero(np.concatenate(([True], key[1:] != key[:-1])))
    mask = np.bitwise_or.reduceat(bits, starts)
    ukey = key[starts]
    return ukey // g.n, ukey % g.n, mask


def num_slice_sets(n: int, sigma: int) -> int:
    return -(-n // sigma)


def vss_partition(set_id, row, mask, n_sets: int, tau: int):
    """Splits the (set, row)-sorted slices into virtual slice sets: the slices of
    each set, in row order, cut into consecutive groups of tau (Section 2.1, rules 1
    and 2), so only a set's last VSS can be short.

    Returns dict with realPtrs (int64[n_sets+1]), virtualToReal (int64[numVSS]) and
    groups: a list of (row int64[], mask uint64[]) per VSS, rows ascending."""
    real_ptrs = [0]
    v2r = []
    groups = []
    bounds = np.searchsorted(set_id, np.arange(n_sets + 1), side="left")
    for s in range(n_sets):
        lo, hi = bounds[s], bounds[s + 1]
        for c in range(lo, hi, tau):
            e = min(hi, c + tau)
            groups.append((row[c:e], mask[c:e]))
            v2r.append(s)
        real_ptrs.append(len(v2r))
    return {"realPtrs": np.array(real_ptrs, np.int64),
            "virtualToReal": np.array(v2r, np.int64),
            "groups": groups}


def placement(k: int, lanes: int):
    """(lane, slot) of the k-th slice of a VSS under column-major placement."""
    return k % lanes, k // lanes


def compression_ratio(m: int, num_slices: int, sigma: int) -> float:
    return 0.0 if num_slices == 0 else m / (num_slices * sigma)


def update_divergence(groups, lanes: int) -> float:
    """Mean over VSSs of the mean (over non-empty slot columns) population standard
    deviation of row IDs in each slot column."""
    per_vss = []
    for rows, _ in groups:
        cols = []
        for c in range(0, len(rows), lanes):
            cols.append(float(np.std(np.asarray(rows[c:c + lanes], dtype=np.float64))))
        if cols:
            per_vss.append(sum(cols) / len(cols))
    return float(np.mean(per_vss)) if per_vss else 0.0


def bvss_bytes_table3(stored_slices: int, num_vss: int, num_sets: int, sigma: int) -> int:
    """Bytes of the static BVSS arrays under the paper's accounting (Table 3):
    rowIds + masks per stored slice, plus virtualToReal and realPtrs entries."""
    return stored_slices * (4 + sigma // 8) + 4 * (num_vss + num_sets)
