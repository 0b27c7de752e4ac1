"""GPU tests of the serving loop: every request's levels equal the oracle's and
equal the request run alone; the HBM budget is never exceeded; overload queues
instead of failing."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")
from paper_2512_21967_amd.serve import Server, poisson_trace, summarize  # noqa: E402


@pytest.fixture(scope="module")
def resident():
    graphs = {"rmat": inputs.rmat_workload(12, 16, seed=3, permute_seed=1),
              "grid": inputs.grid_workload(48, 0.9, seed=2, permute_seed=4)}
    handles = {"rmat": blest.Graph(graphs["rmat"], reorder="compression", window=1024),
               "grid": blest.Graph(graphs["grid"], reorder="bandwidth")}
    return graphs, handles


def src_of(graphs):
    return lambda g, seed, k: inputs.sources(graphs[g], seed=seed, k=k)


@pytest.mark.parametrize("realtime", [True, False])
def test_mixed_trace_matches_oracle_and_alone(resident, realtime):
    graphs, handles = resident
    trace = poisson_trace(7, 4000.0, 120, ["rmat", "grid"], src_of(graphs), k_max=24)
    budget = max(h.footprint(64) for h in handles.values()) * 3
    srv = Server(handles, budget, streams=2)
    reqs = srv.run(trace, realtime=realtime)
    assert srv.peak_bytes <= budget
    assert all(r.done_at is not None and r.latency >= 0 for r in reqs)
    if not realtime:
        assert srv.batches < len(reqs)          # requests were batched together
    for r in reqs:
        got = r.levels.cpu().numpy()
        want = oracle.bfs_multi(graphs[r.graph], r.sources)
        np.testing.assert_array_equal(got, want, err_msg=f"request {r.rid}")
    # the same request alone gives the same levels
    for r in reqs[:10]:
        h = handles[r.graph]
        alone = h.bfs_multi(r.sources) if r.k > 1 else h.bfs(int(r.sources[0])).view(1, -1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(alone.cpu().numpy(), r.levels.cpu().numpy())
    s = summarize(reqs)
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_tight_budget_queues_and_too_small_budget_rejects(resident):
    graphs, handles = resident
    trace = poisson_trace(9, 1e6, 40, ["rmat", "grid"], src_of(graphs), k_max=64)
    budget = max(h.footprint(64) for h in handles.values())   # one full batch at a time
    srv = Server(handles, budget, streams=3)
    reqs = srv.run(trace, realtime=False)
    assert srv.peak_bytes <= budget
    for r in reqs:
        np.testing.assert_array_equal(r.levels.cpu().numpy(), oracle.bfs_multi(graphs[r.graph], r.sources))
    with pytest.raises(ValueError):
        Server(handles, min(h.footprint(1) for h in handles.values()) - 1)
