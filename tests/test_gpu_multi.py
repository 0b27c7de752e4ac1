"""GPU parity of the k-source BFS (``blest_bfs_multi``): row j must equal the
oracle's BFS from sources[j], bit-exact, and equal the single-source GPU run from
the same source.  Covers k = 1..64, repeated sources, every slice width, both
orderings, directed graphs, closed-form families, ragged n and the batched
benchmark graph (R-MAT scale 20, k = 64) on sampled rows."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
import oracle
from tests import families

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")


def run_multi(g, srcs):
    out = g.bfs_multi(np.asarray(srcs, np.uint32))
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name", sorted(families.ALL_FAMILIES))
def test_closed_form_families_all_sources_at_once(name):
    gr, lv = families.ALL_FAMILIES[name]()
    g = blest.Graph(gr, reorder="none")
    srcs = list(range(min(gr.n, 64)))
    got = run_multi(g, srcs)
    for j, s in enumerate(srcs):
        np.testing.assert_array_equal(got[j], lv(s), err_msg=f"{name} row {j} source {s}")


@pytest.mark.parametrize("k", [1, 2, 7, 33, 64])
@pytest.mark.parametrize("sigma", [8, 16, 32])
def test_rmat_k_sources(k, sigma):
    gr = inputs.rmat_workload(12, 16, seed=k + sigma, permute_seed=3)
    g = blest.Graph(gr, sigma=sigma, reorder="none")
    srcs = inputs.sources(gr, seed=k, k=k)
    np.testing.assert_array_equal(run_multi(g, srcs), oracle.bfs_multi(gr, srcs))


def test_repeated_and_isolated_sources():
    gr = inputs.rmat_workload(11, 8, seed=5)
    deg = gr.degrees()
    iso = int(np.flatnonzero(deg == 0)[0])
    s = inputs.sources(gr, seed=1, k=3)
    srcs = [int(s[0]), int(s[0]), iso, int(s[1]), int(s[2]), int(s[1])]
    g = blest.Graph(gr, reorder="none")
    got = run_multi(g, srcs)
    np.testing.assert_array_equal(got, oracle.bfs_multi(gr, srcs))
    np.testing.assert_array_equal(got[0], got[1])


@pytest.mark.parametrize("reorder", ["compression", "bandwidth"])
def test_reordered_multi_matches_single(reorder):
    if reorder == "compression":
        gr = inputs.rmat_workload(12, 16, seed=8, permute_seed=1)
        g = blest.Graph(gr, reorder=reorder, window=1024)
    else:
        gr = inputs.grid_workload(64, 0.9, seed=2, permute_seed=3)
        g = blest.Graph(gr, reorder=reorder)
    srcs = inputs.sources(gr, seed=4, k=16)
    got = run_multi(g, srcs)
    np.testing.assert_array_equal(got, oracle.bfs_multi(gr, srcs))
    for j in (0, 7, 15):
        single = g.bfs(int(srcs[j]))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got[j], single.cpu().numpy())


def test_directed_and_ragged():
    rng = np.random.default_rng(2)
    for n in (1, 3, 65, 1000):
        m = 4 * n
        gr = inputs.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), False)
        g = blest.Graph(gr, reorder="none", slots=1)
        srcs = rng.integers(0, n, min(n, 40))
        np.testing.assert_array_equal(run_multi(g, srcs), oracle.bfs_multi(gr, srcs))


def test_hub_graph():
    star, lv = families.star(20000)
    g = blest.Graph(star, reorder="none", slots=1)
    srcs = [0, 1, 2, 19999]
    got = run_multi(g, srcs)
    for j, s in enumerate(srcs):
        np.testing.assert_array_equal(got[j], lv(s))


def test_repeated_launches_identical():
    gr = inputs.rmat_workload(14, 16, seed=1, permute_seed=2)
    g = blest.Graph(gr, reorder="none")
    srcs = inputs.sources(gr, seed=6, k=64, distinct=True)
    first = run_multi(g, srcs)
    np.testing.assert_array_equal(first[:4], oracle.bfs_multi(gr, srcs[:4]))
    for _ in range(5):
        np.testing.assert_array_equal(run_multi(g, srcs), first)


def test_batched_config_s20_k64_sampled_rows():
    """R-MAT scale 20, edge factor 16, 64 distinct sources in one launch; rows
    sampled against the oracle (the rest checked through invariants)."""
    gr = inputs.rmat_workload(20, 16, seed=1)
    g = blest.Graph(gr, reorder="none")
    srcs = inputs.sources(gr, seed=7, k=64, distinct=True)
    got = run_multi(g, srcs)
    for j in (0, 31, 63):
        np.testing.assert_array_equal(got[j], oracle.bfs(gr, int(srcs[j])))
    # every row: the source has level 0; on a symmetric graph two rows reach
    # either the same component or disjoint ones
    assert np.all(got[np.arange(64), srcs] == 0)
    reached = got >= 0
    for j in range(64):
        assert np.array_equal(reached[j], reached[0]) or not np.any(reached[j] & reached[0])


@pytest.mark.parametrize("slots", [1, 4])
def test_high_diameter_grid(slots):
    """A grid with hundreds of levels (RCM ordering): many k-source levels with
    small frontiers per source."""
    gr = inputs.grid_workload(96, 0.9, seed=4, permute_seed=5)
    g = blest.Graph(gr, reorder="bandwidth", slots=slots)
    srcs = inputs.sources(gr, seed=9, k=40)
    np.testing.assert_array_equal(run_multi(g, srcs), oracle.bfs_multi(gr, srcs))


def _csr_arcs(gr, offset):
    rows = np.repeat(np.arange(gr.n, dtype=np.int64), np.diff(gr.row_ptr.astype(np.int64)))
    return rows + offset, gr.col.astype(np.int64) + offset


def test_levels_switch_between_dense_and_sparse():
    """Two R-MAT blobs joined by a 3,000-vertex path: the blobs' middle levels queue
    many VSSs (full vertex sweep), the path's levels queue one or two (per-vertex
    state bytes), and the k-source call crosses between the two more than once,
    with sources in both blobs and on the path."""
    a = inputs.rmat(12, 8, seed=21)
    b = inputs.rmat(12, 8, seed=22)
    plen = 3000
    base_p, base_b = a.n, a.n + plen
    sa, da = _csr_arcs(a, 0)
    sb, db = _csr_arcs(b, base_b)
    # the path runs from blob a's vertex 0 through base_p .. base_b - 1 into blob b's
    # vertex 0 (R-MAT's vertex 0 has the largest expected degree)
    chain = np.concatenate([[0], np.arange(base_p, base_b), [base_b]]).astype(np.int64)
    ps, pd = chain[:-1], chain[1:]
    n = base_b + b.n
    gr = inputs.from_arcs(n, np.concatenate([sa, sb, ps]), np.concatenate([da, db, pd]), True)
    srcs = np.array([0, 17, base_p + 5, base_p + plen // 2, base_b, base_b + 3, n - 1], np.uint32)
    for reorder in ("none", "compression"):
        g = blest.Graph(gr, reorder=reorder)
        np.testing.assert_array_equal(run_multi(g, srcs), oracle.bfs_multi(gr, srcs), err_msg=reorder)


@pytest.mark.parametrize("ranges", [2, 8, 32])
def test_row_range_partition(ranges):
    """The k-source kernel's own VSS partition cut at row ranges, each workgroup
    pulling one range: R-MAT (dense and sparse levels) and a grid, 64 sources."""
    gr = inputs.rmat_workload(14, 16, seed=ranges, permute_seed=2)
    g = blest.Graph(gr, reorder="none", multi_ranges=ranges)
    st = g.stats()
    assert st["multi_ranges"] == ranges and st["multi_num_vss"] >= st["num_vss"]
    srcs = inputs.sources(gr, seed=5, k=64, distinct=True)
    np.testing.assert_array_equal(run_multi(g, srcs), oracle.bfs_multi(gr, srcs))
    grid = inputs.grid_workload(80, 0.9, seed=ranges, permute_seed=3)
    g = blest.Graph(grid, reorder="bandwidth", multi_ranges=ranges)
    srcs = inputs.sources(grid, seed=6, k=33)
    np.testing.assert_array_equal(run_multi(g, srcs), oracle.bfs_multi(grid, srcs))
    # the single-source kernel keeps its own partition
    s = int(srcs[0])
    np.testing.assert_array_equal(g.bfs(s).cpu().numpy(), oracle.bfs(grid, s))
