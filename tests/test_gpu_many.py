"""GPU parity of the many-graphs launch (``blest_bfs_many`` / ``blest_batch_*``):
every item's levels must equal the oracle's, bit-exact, whatever the mix of sizes,
orderings and sources; a batch replays identically, including under HIP-graph
capture (each replay checked, with eager work between replays)."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
import oracle
from tests import families

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")


def mixed_items():
    graphs = []
    for name in ("path17", "star9", "grid5x7", "hypercube5", "union_paths", "isolated"):
        graphs.append((families.ALL_FAMILIES[name]()[0], "none"))
    rng = np.random.default_rng(4)
    n = 500
    graphs.append((inputs.from_arcs(n, rng.integers(0, n, 1500), rng.integers(0, n, 1500), False), "none"))
    graphs.append((inputs.rmat_workload(12, 16, seed=2, permute_seed=1), "compression"))
    graphs.append((inputs.rmat_workload(16, 16, seed=3), "none"))
    graphs.append((inputs.grid_workload(100, 0.9, seed=1, permute_seed=2), "bandwidth"))
    graphs.append((families.star(30000)[0], "none"))
    return graphs


def test_mixed_graphs_one_launch():
    items = mixed_items()
    handles = [blest.Graph(gr, reorder=ro, window=1024) for gr, ro in items]
    srcs = [int(inputs.sources(gr, seed=i, k=1)[0]) if gr.nnz else 0 for i, (gr, _) in enumerate(items)]
    outs = blest.bfs_many(handles, srcs)
    torch.cuda.synchronize()
    for (gr, _), s, o in zip(items, srcs, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), oracle.bfs(gr, s), err_msg=f"{gr.name} source {s}")


def test_every_source_of_a_family_as_separate_items():
    gr, lv = families.full_grid(6, 9)
    g = blest.Graph(gr, reorder="none")
    srcs = list(range(gr.n))
    outs = blest.bfs_many([g] * gr.n, srcs)
    torch.cuda.synchronize()
    for s, o in zip(srcs, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), lv(s))


def test_batch_replays_and_graph_capture():
    rec = inputs.many_graphs_recipe(24, base_seed=500, scale_range=(10, 13))
    graphs = [inputs.rmat(s, ef, seed) for s, ef, seed in rec]
    handles = [blest.Graph(gr, reorder="none") for gr in graphs]
    srcs = [int(inputs.sources(gr, seed=1, k=1)[0]) for gr in graphs]
    want = [oracle.bfs(gr, s) for gr, s in zip(graphs, srcs)]
    batch = blest.Batch(handles, srcs)
    for _ in range(2):
        for o in batch.outs:
            o.fill_(7)
        batch.run()
        torch.cuda.synchronize()
        for o, w in zip(batch.outs, want):
            np.testing.assert_array_equal(o.cpu().numpy(), w)
    cg = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(cg, stream=stream):
            batch.run(stream=stream)
    torch.cuda.synchronize()
    for _ in range(3):
        for o in batch.outs:
            o.fill_(-5)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        for o, w in zip(batch.outs, want):
            np.testing.assert_array_equal(o.cpu().numpy(), w)
        # eager work between replays
        handles[0].bfs(srcs[0])
        torch.cuda.synchronize()
    batch.close()


def test_many_graphs_config_sample():
    """A 32-graph slice of the 256-graph configuration (scale 10..16, edge factor
    8..32), every item checked."""
    rec = inputs.many_graphs_recipe(256, base_seed=1000)[:32]
    graphs = [inputs.rmat(s, ef, seed) for s, ef, seed in rec]
    handles = [blest.Graph(gr, reorder="none") for gr in graphs]
    srcs = [int(inputs.sources(gr, seed=seed, k=1)[0]) for gr, (_, _, seed) in zip(graphs, rec)]
    outs = blest.bfs_many(handles, srcs)
    torch.cuda.synchronize()
    for gr, s, o in zip(graphs, srcs, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), oracle.bfs(gr, s))


def test_too_large_graph_rejected():
    gr = inputs.from_arcs(131073, [0], [1], True)
    g = blest.Graph(gr, reorder="none")
    with pytest.raises(blest.BlestError):
        blest.bfs_many([g], [0])
