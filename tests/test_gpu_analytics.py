"""GPU parity of the multi-source analytics (``blest_level_stats`` and the sweeps on
``blest_bfs_multi``) against ``oracle.analytics``: reached counts, level sums,
eccentricities and farthest vertices bit-exact, closeness bit-exact (both sides
divide the same two integers in double precision).  Covers closed-form families,
empty and all-unreached rows, n = 0 and 1, ragged n spanning many workgroups, k up
to 64, the batched benchmark graph (R-MAT scale 20, k = 64) on sampled rows and
the diameter sweeps."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
import oracle
from oracle import analytics
from tests import families

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")

KEYS = ("reached", "total", "ecc", "far", "closeness")


def gpu_stats(levels_np):
    t = torch.from_numpy(np.ascontiguousarray(levels_np, np.int32)).cuda()
    st = blest.level_stats(t)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in st.items()}


def assert_same(got, want, rows=None, what=""):
    for key in KEYS:
        g = np.asarray(got[key])
        w = np.asarray(want[key])
        if rows is not None:
            g = g[rows]
        np.testing.assert_array_equal(g.astype(np.float64 if key == "closeness" else np.int64),
                                      w.astype(np.float64 if key == "closeness" else np.int64),
                                      err_msg=f"{what} {key}")


@pytest.mark.parametrize("name", sorted(families.ALL_FAMILIES))
def test_families_all_sources(name):
    gr, _ = families.ALL_FAMILIES[name]()
    g = blest.Graph(gr, reorder="none")
    srcs = list(range(min(gr.n, 64)))
    got = g.source_stats(srcs)
    want = analytics.source_stats(oracle.bfs_multi(gr, srcs))
    assert_same(got, want, what=name)


@pytest.mark.parametrize("k,n", [(1, 1), (3, 1000), (5, 3_000_017), (64, 4097)])
def test_synthetic_level_arrays(k, n):
    rng = np.random.default_rng(k * 31 + n)
    lv = rng.integers(-1, 40, size=(k, n), dtype=np.int32)
    lv[0, :] = -1                      # an empty row
    if k > 2:
        lv[2, :] = rng.integers(-1, 2, size=n)
        lv[2, n - 1] = 1000            # the maximum at the ragged tail
    assert_same(gpu_stats(lv), analytics.source_stats(lv), what=f"k={k} n={n}")


def test_zero_length_rows():
    t = torch.empty((4, 0), dtype=torch.int32, device="cuda")
    st = blest.level_stats(t)
    torch.cuda.synchronize()
    assert st["reached"].cpu().tolist() == [0] * 4
    assert st["ecc"].cpu().tolist() == [-1] * 4
    assert st["far"].cpu().tolist() == [0xFFFFFFFF] * 4
    assert st["closeness"].cpu().tolist() == [0.0] * 4


def test_rmat_and_grid_parity():
    for gr, ro, seed in ((inputs.rmat_workload(14, 16, seed=5, permute_seed=6), "compression", 1),
                         (inputs.grid_workload(96, 0.9, seed=3, permute_seed=4), "bandwidth", 2)):
        g = blest.Graph(gr, reorder=ro)
        srcs = inputs.sources(gr, seed=seed, k=40)
        assert_same(g.source_stats(srcs), analytics.source_stats(oracle.bfs_multi(gr, srcs)), what=gr.name)


def test_batched_benchmark_graph_sampled_rows():
    """R-MAT scale 20 with the benchmark's 64 sources in one launch; the oracle
    computes three of the rows."""
    gr = inputs.rmat_workload(20, 16, seed=1)
    srcs = inputs.sources(gr, seed=7, k=64, distinct=True)
    g = blest.Graph(gr, reorder="none")
    got = g.source_stats(srcs)
    rows = [0, 31, 63]
    want = analytics.source_stats(np.stack([oracle.bfs(gr, int(srcs[j])) for j in rows]))
    assert_same(got, want, rows=rows, what="rmat20 k=64")


@pytest.mark.parametrize("case", ["path", "grid", "hypercube", "union", "rmat"])
def test_diameter_sweeps_match_oracle(case):
    if case == "path":
        gr, _ = families.path(301)
        srcs = [150, 7]
    elif case == "grid":
        gr, _ = families.full_grid(40, 57)
        srcs = [1000, 5]
    elif case == "hypercube":
        gr, _ = families.hypercube(7)
        srcs = [0, 77]
    elif case == "union":
        gr, _ = families.disjoint_union_paths(60, 90)
        srcs = [3, 100]
    else:
        gr = inputs.rmat_workload(13, 16, seed=9, permute_seed=10)
        srcs = list(inputs.sources(gr, seed=4, k=16))
    g = blest.Graph(gr, reorder="none")
    got = g.diameter_bounds(srcs, sweeps=3)
    want = analytics.diameter_bounds(gr, srcs, sweeps=3)
    assert got == want
    if case == "path":
        assert got[:2] == (300, 300)
    if case == "grid":
        assert got[0] == 40 + 57 - 2
