"""GPU parity of the single-source BFS (``blest_bfs``) with the oracle, through the
C-ABI.  Levels must be bit-exact; parents must pass the Graph500-style checks.
Covers both update schemes (Algorithm 2 eager, Algorithm 3 lazy), every slice width
and slot count, the two orderings, tiny closed-form families, ragged and degenerate
inputs, a hub whose slice set spans many VSSs, directed graphs (pull direction),
and repeated runs (no races)."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
import oracle
from tests import families

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")


def run(g, s, parents=False):
    out = g.bfs(int(s), parents=parents)
    torch.cuda.synchronize()
    if parents:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def check_sources(gr, g, srcs, with_parents=False):
    for s in srcs:
        s = int(s)
        want = oracle.bfs(gr, s)
        if with_parents:
            got, par = run(g, s, parents=True)
            np.testing.assert_array_equal(got, want, err_msg=f"{gr.name or 'graph'} source {s}")
            assert oracle.validate_tree(gr, s, want, par) == 0, f"bad parents from source {s}"
        else:
            got = run(g, s)
            np.testing.assert_array_equal(got, want, err_msg=f"{gr.name or 'graph'} source {s}")


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
@pytest.mark.parametrize("name", sorted(families.ALL_FAMILIES))
def test_closed_form_families_every_source(name, update):
    gr, lv = families.ALL_FAMILIES[name]()
    g = blest.Graph(gr, update=update, reorder="none")
    for s in range(gr.n):
        np.testing.assert_array_equal(run(g, s), lv(s), err_msg=f"{name} source {s} ({update})")


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
@pytest.mark.parametrize("sigma,slots", [(8, 1), (8, 2), (8, 4), (8, 8), (16, 4), (32, 2)])
def test_rmat_widths_and_slots(sigma, slots, update):
    gr = inputs.rmat_workload(13, 16, seed=sigma * 10 + slots, permute_seed=1)
    g = blest.Graph(gr, sigma=sigma, slots=slots, update=update, reorder="none")
    check_sources(gr, g, inputs.sources(gr, seed=3, k=4))


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
@pytest.mark.parametrize("reorder", ["compression", "bandwidth"])
def test_reordered_graphs_map_back(reorder, update):
    if reorder == "compression":
        gr = inputs.rmat_workload(12, 16, seed=4, permute_seed=2)
        kw = dict(window=1024)
    else:
        gr = inputs.grid_workload(96, 0.9, seed=2, permute_seed=5)
        kw = {}
    g = blest.Graph(gr, reorder=reorder, update=update, **kw)
    check_sources(gr, g, inputs.sources(gr, seed=8, k=4))


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
def test_parents_pass_graph500_checks(update):
    gr = inputs.rmat_workload(12, 16, seed=6, permute_seed=3)
    g = blest.Graph(gr, update=update, reorder="compression", window=512)
    check_sources(gr, g, inputs.sources(gr, seed=2, k=3), with_parents=True)
    grid = inputs.grid_workload(40, 0.9, seed=1, permute_seed=2)
    g = blest.Graph(grid, update=update)
    check_sources(grid, g, inputs.sources(grid, seed=2, k=2), with_parents=True)


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
def test_directed_graphs_follow_out_edges(update):
    rng = np.random.default_rng(11)
    for n in (2, 31, 33, 257, 3000):
        m = 3 * n
        gr = inputs.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), False)
        g = blest.Graph(gr, update=update, reorder="none", slots=1)
        check_sources(gr, g, range(0, n, max(1, n // 5)))


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
def test_degenerate_inputs(update):
    # one vertex, no arcs
    one = inputs.from_arcs(1, [], [], False)
    g = blest.Graph(one, update=update, reorder="none")
    np.testing.assert_array_equal(run(g, 0), [0])
    # isolated source inside a set that has VSSs
    gr = inputs.from_arcs(40, [1, 2, 3, 9], [2, 3, 4, 10], True)
    g = blest.Graph(gr, update=update, reorder="none")
    for s in (0, 1, 5, 9, 39):
        np.testing.assert_array_equal(run(g, s), oracle.bfs(gr, s))
    # hub: the centre's slice set spans many VSSs
    star, lv = families.star(20000)
    g = blest.Graph(star, update=update, reorder="none", slots=1)
    for s in (0, 1, 19999):
        np.testing.assert_array_equal(run(g, s), lv(s))


def test_repeated_runs_identical():
    gr = inputs.rmat_workload(14, 16, seed=9, permute_seed=4)
    for update in ("eager", "lazy", "adaptive"):
        g = blest.Graph(gr, update=update, reorder="none")
        s = int(inputs.sources(gr, seed=1, k=1)[0])
        want = oracle.bfs(gr, s)
        for _ in range(20):
            np.testing.assert_array_equal(run(g, s), want)


def test_launch_shapes():
    """Workgroup shapes, including one asking for two 1024-thread workgroups per CU:
    every persistent kernel here allocates more than 96 scalar registers (at most 7
    wavefronts per SIMD), so that request is clamped to one workgroup per CU."""
    gr = inputs.rmat_workload(12, 16, seed=2, permute_seed=7)
    srcs = inputs.sources(gr, seed=5, k=2)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for block, per_cu in ((64, 1), (256, 1), (1024, 1), (256, 4), (512, 2), (1024, 2)):
        for update in ("eager", "lazy"):
            g = blest.Graph(gr, update=update, reorder="none", block=block, blocks_per_cu=per_cu)
            st = g.stats()
            print(f"shape {block}x{per_cu} {update}: vgprs {st['kernel_vgprs']} runtime "
                  f"{st['blocks_per_cu_runtime']} own {st['blocks_per_cu_own']} grid {st['grid']}", flush=True)
            assert st["grid"] == cus * min(per_cu, st["blocks_per_cu_own"], st["blocks_per_cu_runtime"])
            assert st["blocks_per_cu_own"] * block <= 7 * 4 * 64
            check_sources(gr, g, srcs)


def test_streams_and_async():
    gr = inputs.rmat_workload(12, 16, seed=3, permute_seed=1)
    g = blest.Graph(gr, reorder="none")
    srcs = [int(x) for x in inputs.sources(gr, seed=4, k=6)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = []
    for i, s in enumerate(srcs):
        st = streams[i % 3]
        with torch.cuda.stream(st):
            outs.append(g.bfs(s, stream=st))
    torch.cuda.synchronize()
    for s, o in zip(srcs, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), oracle.bfs(gr, s))


def test_full_size_s16_config():
    """R-MAT scale 16, edge factor 16, plain ordering (the small benchmark config)."""
    gr = inputs.rmat_workload(16, 16, seed=1)
    for update in ("eager", "lazy", "adaptive"):
        g = blest.Graph(gr, reorder="none", update=update)
        check_sources(gr, g, inputs.sources(gr, seed=1, k=3))


@pytest.mark.parametrize("ranges", [1, 2, 8, 32])
@pytest.mark.parametrize("update", ["lazy", "eager", "adaptive"])
def test_row_ranges(ranges, update):
    """VSSs cut at row-range boundaries; the lazy kernel keeps each workgroup's
    range of visited bits in LDS."""
    gr = inputs.rmat_workload(14, 16, seed=ranges, permute_seed=3)
    g = blest.Graph(gr, update=update, reorder="none", ranges=ranges)
    assert g.stats()["nranges"] == ranges
    check_sources(gr, g, inputs.sources(gr, seed=ranges, k=3))


def test_lazy_with_partial_lds_cache():
    """A graph whose visited bitmap is larger than the LDS cache: the lowest rows
    are checked in LDS, the others in global memory (S20, 64 KiB cache)."""
    gr = inputs.rmat_workload(20, 4, seed=2, permute_seed=1)
    g = blest.Graph(gr, update="lazy", reorder="none", ranges=1, lds_kib=64)
    st = g.stats()
    assert st["hubs_sorted"] == 1 and st["lds_bytes"] * 8 == gr.n // 2
    check_sources(gr, g, inputs.sources(gr, seed=1, k=2))
    g.configure(update="eager")
    check_sources(gr, g, inputs.sources(gr, seed=2, k=1))


@pytest.mark.parametrize("lds_kib", [1, 4, None])
@pytest.mark.parametrize("ranges", [1, 4])
@pytest.mark.parametrize("hubs", ["on", "off"])
def test_lds_cache_sizes(lds_kib, ranges, hubs):
    """Small LDS caches (1 KiB = 8192 rows, 4 KiB) so that most levels use the cache
    and many rows fall outside it; None = no cache (global checks only)."""
    gr = inputs.rmat_workload(15, 16, seed=7, permute_seed=8)
    g = blest.Graph(gr, update="lazy", reorder="none", ranges=ranges, hubs=hubs, lds_kib=lds_kib)
    st = g.stats()
    assert st["lds_bytes"] == (0 if lds_kib is None else min(lds_kib * 1024, st["range_len"] // 8))
    assert st["hubs_sorted"] == (hubs == "on")
    check_sources(gr, g, inputs.sources(gr, seed=ranges, k=3))


def test_full_size_s22_config_sampled_sources():
    """R-MAT scale 22, edge factor 16, labels permuted, Algorithm 1 ordering: the
    benchmark configuration, in its default launch shape, on sampled sources."""
    gr = inputs.rmat_workload(22, 16, seed=1, permute_seed=2)
    g = blest.Graph(gr, reorder="compression")
    st = g.stats()
    assert st["update_used"] == "lazy" and st["nranges"] == 1 and st["hubs_sorted"] == 1
    assert st["prepass_used"] == 1 and st["window_used"] == 4096
    assert st["lds_bytes"] == 128 * 1024 and st["lds_bytes"] * 8 < gr.n
    check_sources(gr, g, inputs.sources(gr, seed=3, k=64)[:2])


@pytest.mark.parametrize("prepass,window", [("shingle", 0), ("shingle", 1 << 16), ("off", 0)])
def test_shingle_prepass_orderings(prepass, window):
    """The shingle pre-pass before Algorithm 1 (default window and a large one) and
    Algorithm 1 alone: every ordering is a relabelling, so levels in the caller's
    IDs must match the oracle on every source."""
    gr = inputs.rmat_workload(14, 16, seed=21, permute_seed=22)
    g = blest.Graph(gr, reorder="compression", prepass=prepass, window=window)
    st = g.stats()
    assert st["prepass_used"] == (prepass == "shingle")
    assert st["window_used"] == (window or (4096 if prepass == "shingle" else 65536))
    check_sources(gr, g, inputs.sources(gr, seed=23, k=6))


@pytest.mark.parametrize("case,max_grid,update", [("grid", 32, "eager"), ("grid", 64, "adaptive"),
                                                   ("rmat", 8, "lazy"), ("rmat", 1, "auto")])
def test_capped_grid(case, max_grid, update):
    """A single-source launch capped to a few workgroups (cheaper grid barriers on
    high-diameter graphs) gives the same levels."""
    if case == "grid":
        gr = inputs.grid_workload(200, 0.9, seed=31, permute_seed=32)
        g = blest.Graph(gr, reorder="bandwidth", update=update, max_grid=max_grid)
    else:
        gr = inputs.rmat_workload(13, 16, seed=33, permute_seed=34)
        g = blest.Graph(gr, reorder="compression", update=update, max_grid=max_grid)
    assert g.stats()["grid"] == max_grid
    check_sources(gr, g, inputs.sources(gr, seed=35, k=4))


def _csr_arcs(gr, offset):
    rows = np.repeat(np.arange(gr.n, dtype=np.int64), np.diff(gr.row_ptr.astype(np.int64)))
    return rows + offset, gr.col.astype(np.int64) + offset


@pytest.mark.parametrize("eager_max", [1, 3, 40, 400, 1 << 30])
@pytest.mark.parametrize("lds_kib", [0, None])
def test_adaptive_switches_between_schemes(eager_max, lds_kib):
    """Two R-MAT blobs joined by a 2,000-vertex path: the blobs' middle levels queue
    many VSSs, the path's levels one or two, so with thresholds between those sizes
    the BFS switches between eager and lazy levels several times (eager after
    eager, eager after lazy, lazy after eager, lazy after lazy); 1 and 2^30 make
    every level lazy or eager."""
    a = inputs.rmat(13, 8, seed=31)
    b = inputs.rmat(12, 16, seed=32)
    plen = 2000
    base_p, base_b = a.n, a.n + plen
    sa, da = _csr_arcs(a, 0)
    sb, db = _csr_arcs(b, base_b)
    chain = np.concatenate([[0], np.arange(base_p, base_b), [base_b]]).astype(np.int64)
    n = base_b + b.n
    gr = inputs.from_arcs(n, np.concatenate([sa, sb, chain[:-1]]), np.concatenate([da, db, chain[1:]]), True)
    g = blest.Graph(gr, update="adaptive", reorder="none", eager_max=eager_max, lds_kib=lds_kib)
    st = g.stats()
    assert st["update_used"] == "adaptive" and st["eager_max"] == eager_max
    srcs = [0, 17, base_p + 5, base_p + plen // 2, base_b, base_b + 3, n - 1]
    check_sources(gr, g, srcs)
    out = torch.empty(gr.n, dtype=torch.int32, device="cuda")
    for s in srcs[:3]:  # the allocation-free entry point runs the same scheme
        g.bfs_noalloc(s, out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.bfs(gr, s))


def test_adaptive_default_threshold_on_rmat_and_grid():
    gr = inputs.rmat_workload(17, 16, seed=5, permute_seed=6)
    g = blest.Graph(gr, update="adaptive", reorder="compression", window=4096)
    assert g.stats()["eager_max"] == max(1, g.stats()["num_vss"] // 32)
    check_sources(gr, g, inputs.sources(gr, seed=4, k=4), with_parents=True)
    grid = inputs.grid_workload(128, 0.9, seed=5, permute_seed=6)
    g = blest.Graph(grid, update="adaptive", reorder="bandwidth")
    check_sources(grid, g, inputs.sources(grid, seed=4, k=3))


def test_occupancy_answer_and_scalar_registers():
    """The eager kernel at sigma 8, one slot, group depth 1 uses 64 vector registers,
    which alone would allow 8 wavefronts per SIMD; its scalar registers allow 7.  The
    grid asked for as two 1024-thread workgroups per CU is held to one (the
    runtime's answer is printed for the record)."""
    gr = inputs.rmat_workload(12, 16, seed=2, permute_seed=7)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    g = blest.Graph(gr, update="eager", reorder="none", slots=1, group=1, block=1024, blocks_per_cu=2)
    st = g.stats()
    print(f"eager sigma 8 slots 1 group 1: vgprs {st['kernel_vgprs']} runtime {st['blocks_per_cu_runtime']} "
          f"own {st['blocks_per_cu_own']} grid {st['grid']}", flush=True)
    assert st["blocks_per_cu_own"] == 1 and st["grid"] == cus
    check_sources(gr, g, inputs.sources(gr, seed=5, k=2))
