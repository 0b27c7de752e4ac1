"""Pins for the BVSS oracle (``oracle.bvss``): the Figure 1 worked example, the
97-slice placement example (Section 2.1.2), Table 3's accounting relations, closed
forms of the compression ratio, brute-force slices from a dense matrix, and
hand-computed update divergences."""
from __future__ import annotations

import csv
import json
import math
import os

import numpy as np
import pytest

import inputs
from oracle import bvss
from tests import families

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def drawn_to_bits(s: str) -> int:
    """Figures draw column 0 on the left: character j is bit j."""
    return sum(1 << j for j, ch in enumerate(s) if ch == "1")


def fig1():
    with open(os.path.join(GOLDEN, "fig1_bvss.json")) as f:
        fx = json.load(f)
    src, dst = zip(*fx["arcs"])
    g = inputs.from_arcs(fx["n"], src, dst, False)
    return fx, g


def test_fig1_vss_ownership():
    fx, g = fig1()
    sid, row, mask = bvss.slices(g, fx["sigma"])
    part = bvss.vss_partition(sid, row, mask, bvss.num_slice_sets(g.n, fx["sigma"]), fx["tau"])
    assert part["realPtrs"].tolist() == fx["realPtrs"]
    assert part["virtualToReal"].tolist() == fx["virtualToReal"]
    sizes = [len(r) for r, _ in part["groups"]]
    assert all(sizes[v] == fx["tau"] for v in fx["full_vss"])
    assert all(sizes[v] < fx["tau"] for v in fx["padded_vss"])
    # padded VSSs are exactly the short last VSSs of their sets
    last_of_set = {int(part["realPtrs"][s + 1]) - 1 for s in range(3)}
    assert set(fx["padded_vss"]) <= last_of_set


def test_fig1_row3_mask_and_pull():
    fx, g = fig1()
    sigma = fx["sigma"]
    sid, row, mask = bvss.slices(g, sigma)
    m3 = int(mask[(sid == 2) & (row == 3)][0])
    assert m3 == drawn_to_bits(fx["row3_set2_mask_drawn"])
    alpha = drawn_to_bits(fx["set2_frontier_drawn"])
    part = bvss.vss_partition(sid, row, mask, 3, fx["tau"])
    hits = sorted(int(u) for v in fx["active_vss"] for u, m in zip(*part["groups"][v]) if int(m) & alpha)
    assert hits == fx["expected_hits"]
    pushed = sorted({p for u in hits for p in range(part["realPtrs"][u // sigma], part["realPtrs"][u // sigma + 1])})
    assert pushed == fx["expected_push"]


def test_tau_rule_and_97_slice_placement():
    # Section 2.1: tau = WARP_SIZE * slicesPerThread, slicesPerThread = 32 / sigma.
    sigma = 8
    slices_per_thread = 32 // sigma
    tau = 32 * slices_per_thread
    assert (slices_per_thread, tau) == (4, 128)
    # Section 2.1.2: 97 sorted slices under column-major placement keep all 32
    # lanes busy; the row-major packing of the prior layout leaves lanes idle.
    lanes_used = {bvss.placement(k, 32)[0] for k in range(97)}
    assert lanes_used == set(range(32))
    assert max(bvss.placement(k, 32)[1] for k in range(97)) == 3
    row_major_threads = {k // slices_per_thread for k in range(97)}
    assert len(row_major_threads) == 25


def read_table3():
    with open(os.path.join(GOLDEN, "table3_bvss.csv")) as f:
        return list(csv.DictReader(line for line in f if not line.startswith("#")))


def test_table3_byte_accounting():
    for r in read_table3():
        b = bvss.bvss_bytes_table3(int(r["slices"]), int(r["vss"]), int(r["slice_sets"]), 8)
        # the printed GB value is the byte count in units of 1e9, truncated to 2 decimals
        assert math.floor(b / 1e7) == round(float(r["mem_bvss"]) * 100), r["graph"]


def test_table3_bits_pin_sigma_8():
    for r in read_table3():
        assert int(r["unpadded_slices"]) * 8 == int(r["conn_bits"]), r["graph"]
        assert int(r["slices"]) >= int(r["unpadded_slices"])
        # rule 1 of Section 2.1 with tau = 128: no VSS holds more than 128 slices
        assert int(r["slices"]) <= int(r["vss"]) * 128, r["graph"]
        # every set with slices has a VSS
        assert int(r["vss"]) >= -(-int(r["unpadded_slices"]) // 128)


def test_compression_closed_forms():
    sigma = 8
    # directed cycle: every vertex has one in-neighbour -> one bit per slice
    n = 64
    g = inputs.from_arcs(n, np.arange(n), (np.arange(n) + 1) % n, False)
    sid, row, mask = bvss.slices(g, sigma)
    assert bvss.compression_ratio(g.nnz, len(sid), sigma) == pytest.approx(1 / sigma)
    # complete bipartite between two sigma-aligned sides -> full masks
    src, dst = zip(*[(u, 8 + v) for u in range(8) for v in range(8)])
    g = inputs.from_arcs(16, src, dst, True)
    sid, row, mask = bvss.slices(g, sigma)
    assert len(sid) == 16 and np.all(mask == 0xFF)
    assert bvss.compression_ratio(g.nnz, len(sid), sigma) == 1.0


@pytest.mark.parametrize("sigma", [1, 3, 8, 16])
def test_slices_match_dense_definition(sigma):
    rng = np.random.default_rng(sigma)
    for trial in range(20):
        n = int(rng.integers(1, 40))
        adj = (rng.random((n, n)) < 0.15).astype(np.uint8)
        np.fill_diagonal(adj, 0)
        g = families.small_dense_csr(n, adj)
        sid, row, mask = bvss.slices(g, sigma)
        A = adj.T  # A[u][v] = arc v -> u
        expect = []
        for i in range(-(-n // sigma)):
            for u in range(n):
                m = 0
                for j in range(sigma):
                    c = sigma * i + j
                    if c < n and A[u, c]:
                        m |= 1 << j
                if m:
                    expect.append((i, u, m))
        got = list(zip(sid.tolist(), row.tolist(), [int(x) for x in mask]))
        assert got == expect
        assert sum(bin(m).count("1") for *_, m in got) == int(g.row_ptr[-1])


def test_update_divergence_hand_values():
    groups = [(np.array([0, 2]), None)]
    assert bvss.update_divergence(groups, 32) == pytest.approx(1.0)
    groups = [(np.array([0, 2]), None), (np.array([10]), None)]
    assert bvss.update_divergence(groups, 32) == pytest.approx(0.5)
    # lanes = 2: columns {0, 4} and {10} -> (2 + 0) / 2
    groups = [(np.array([0, 4, 10]), None)]
    assert bvss.update_divergence(groups, 2) == pytest.approx(1.0)


def test_vss_partition_rules_on_random_graph():
    g = inputs.rmat(10, 16, seed=3)
    sigma, tau = 8, 128
    sid, row, mask = bvss.slices(g, sigma)
    n_sets = bvss.num_slice_sets(g.n, sigma)
    part = bvss.vss_partition(sid, row, mask, n_sets, tau)
    rp, v2r = part["realPtrs"], part["virtualToReal"]
    assert rp[0] == 0 and rp[-1] == len(v2r) and np.all(np.diff(rp) >= 0)
    for s in range(n_sets):
        cnt = int(np.sum(sid == s))
        assert rp[s + 1] - rp[s] == -(-cnt // tau)
        assert np.all(v2r[rp[s]:rp[s + 1]] == s)
    assert sum(len(r) for r, _ in part["groups"]) == len(sid)
    for r, _ in part["groups"]:
        assert 1 <= len(r) <= tau and np.all(np.diff(r) > 0)
