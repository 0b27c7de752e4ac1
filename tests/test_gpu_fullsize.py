"""GPU parity at the full sizes of the benchmark workloads, every output checked
against the oracle element by element (levels are integers: tolerance 0), in the
launch configuration the benchmark times:

  * R-MAT scale 22, edge factor 16, permuted labels, Algorithm 1 ordering: all 64
    single-source BFSs;
  * R-MAT scale 20, edge factor 16: all 64 rows of one k = 64 launch;
  * 4096 x 4096 grid, p = 0.9, permuted labels, RCM: all 16 single-source BFSs
    (thousands of levels each);
  * 256 R-MAT graphs of scale 10..16 in one graph-captured launch: every graph,
    on two replays;
  * the serving graphs (R-MAT scale 18, R-MAT scale 22, 2048 x 2048 grid) under a
    Poisson request trace: every request.

The oracle runs on host threads (tests/oracle_pool.py), so each test stays well
inside its time limit."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
from tests import oracle_pool

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def s22():
    gr = inputs.rmat_workload(22, 16, seed=1, permute_seed=2)
    g = blest.Graph(gr, reorder="compression")
    return gr, g


def test_s22_all_64_sources(s22):
    """Every source under the static rule (lazy here) and under the adaptive scheme."""
    gr, g = s22
    st = g.stats()
    assert st["update_used"] == "lazy" and st["hubs_sorted"] == 1
    srcs = inputs.sources(gr, seed=3, k=64)
    say(f"S22: n={gr.n} arcs={gr.nnz} VSS={st['num_vss']} grid={st['grid']}x{st['block']}")
    want = oracle_pool.rows(gr, srcs)
    out = torch.empty(gr.n, dtype=torch.int32, device="cuda")
    for update in ("auto", "adaptive"):
        g.configure(update=update)
        for j, s in enumerate(srcs):
            g.bfs(int(s), levels=out)
            got = out.cpu().numpy()
            np.testing.assert_array_equal(got, want[j], err_msg=f"S22 {update} source {int(s)} (#{j})")
    g.configure(update="auto")


def test_s20_k64_all_rows():
    """Every row, with the k-source kernel on the base VSS partition and on its own
    partition cut at 8 row ranges."""
    gr = inputs.rmat_workload(20, 16, seed=1)
    srcs = inputs.sources(gr, seed=7, k=64, distinct=True)
    want = oracle_pool.rows(gr, srcs)
    for ranges in (1, 8):
        g = blest.Graph(gr, reorder="none", multi_ranges=ranges)
        say(f"S20 x 64: n={gr.n} arcs={gr.nnz} ranges {ranges}")
        got = g.bfs_multi(srcs).cpu().numpy()
        for j in range(64):
            np.testing.assert_array_equal(got[j], want[j], err_msg=f"S20 ranges {ranges} row {j} source {int(srcs[j])}")
        g.close()


def test_grid4096_all_16_sources():
    gr = inputs.grid_workload(4096, 0.9, seed=3, permute_seed=4)
    g = blest.Graph(gr, reorder="bandwidth")
    st = g.stats()
    assert st["reorder_used"] == "bandwidth"
    srcs = inputs.sources(gr, seed=5, k=16)
    say(f"grid 4096^2: n={gr.n} arcs={gr.nnz} update={st['update_used']}")
    want = oracle_pool.rows(gr, srcs)
    out = torch.empty(gr.n, dtype=torch.int32, device="cuda")
    for update in ("auto", "adaptive"):
        g.configure(update=update)
        for j, s in enumerate(srcs):
            g.bfs(int(s), levels=out)
            np.testing.assert_array_equal(out.cpu().numpy(), want[j], err_msg=f"grid {update} source {int(s)} (#{j})")
    assert want.max() > 4000  # thousands of levels


def test_many256_all_graphs_captured():
    rec = inputs.many_graphs_recipe(256, base_seed=1000)
    graphs = [inputs.rmat(s, ef, seed) for s, ef, seed in rec]
    handles = [blest.Graph(gr, reorder="none") for gr in graphs]
    srcs = [int(inputs.sources(gr, seed=seed, k=1)[0]) for gr, (_, _, seed) in zip(graphs, rec)]
    say(f"many256: {sum(gr.n for gr in graphs)} vertices, {sum(gr.nnz for gr in graphs)} arcs")
    want = oracle_pool.each(zip(graphs, srcs))
    batch = blest.Batch(handles, srcs)
    stream = torch.cuda.Stream()
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(cg, stream=stream):
            batch.run(stream=stream)
    torch.cuda.synchronize()
    for rep in range(2):
        for o in batch.outs:
            o.fill_(-7)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(batch.outs, want)):
            np.testing.assert_array_equal(o.cpu().numpy(), w, err_msg=f"replay {rep} graph {i} ({graphs[i].name})")
    batch.close()
    for h in handles:
        h.close()


def test_serving_graphs_every_request(s22):
    from paper_2512_21967_amd.serve import Server, poisson_trace
    gr22, g22 = s22
    graphs = {"rmat18": inputs.rmat_workload(18, 16, seed=11, permute_seed=12),
              "rmat22": gr22,
              "grid2048": inputs.grid_workload(2048, 0.9, seed=3, permute_seed=4)}
    handles = {"rmat18": blest.Graph(graphs["rmat18"]), "rmat22": g22, "grid2048": blest.Graph(graphs["grid2048"])}
    for name, h in handles.items():
        st = h.stats()
        say(f"{name}: {st['reorder_used']}/{st['update_used']}")
    src_of = lambda g, seed, k: inputs.sources(graphs[g], seed=seed, k=k)
    trace = poisson_trace(5, 200.0, 24, list(graphs), src_of, k_max=32)
    budget = 16 << 30
    srv = Server(handles, budget)
    pairs, got = [], []

    def take(r):
        lv = r.levels.cpu().numpy()
        for j in range(r.k):
            pairs.append((graphs[r.graph], int(r.sources[j])))
            got.append((r.rid, r.graph, j, lv[j]))

    reqs = srv.run(trace, keep=False, on_done=take)
    srv.close()
    assert all(r.done_at is not None for r in reqs) and srv.peak_bytes <= budget
    want = oracle_pool.each(pairs)
    for (rid, name, j, lv), w in zip(got, want):
        np.testing.assert_array_equal(lv, w, err_msg=f"request {rid} ({name}) row {j}")
    say(f"{len(reqs)} requests, {len(got)} rows")
