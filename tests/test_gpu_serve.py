"""GPU tests of the continuous-batching server (blest_server_* through the serving
loop): every request's levels equal the oracle's and the same request run alone;
requests that arrive while others run are admitted into the running sweep (their
device lifetimes overlap); the HBM budget bounds both the server's ledger and the
device memory PyTorch actually handed out; the launch ends when idle and starts
again on the next request."""
from __future__ import annotations

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")
from paper_2512_21967_amd.serve import Server, overlapping_pairs, poisson_trace, summarize  # noqa: E402


@pytest.fixture(scope="module")
def resident():
    graphs = {"rmat": inputs.rmat_workload(12, 16, seed=3, permute_seed=1),
              "grid": inputs.grid_workload(48, 0.9, seed=2, permute_seed=4),
              "small": inputs.rmat(9, 8, seed=5)}
    handles = {"rmat": blest.Graph(graphs["rmat"], reorder="compression", window=1024),
               "grid": blest.Graph(graphs["grid"], reorder="bandwidth"),
               "small": blest.Graph(graphs["small"], reorder="none")}
    return graphs, handles


def src_of(graphs):
    return lambda g, seed, k: inputs.sources(graphs[g], seed=seed, k=k)


def to_host(r):
    r.host = r.levels.cpu().numpy()


@pytest.mark.parametrize("realtime", [True, False])
def test_mixed_trace_matches_oracle_and_alone(resident, realtime):
    graphs, handles = resident
    trace = poisson_trace(7, 3000.0, 120, list(graphs), src_of(graphs), k_max=24)
    budget = 64 << 20
    srv = Server(handles, budget)
    print(f"serve realtime={realtime}: {len(trace)} requests", flush=True)
    reqs = srv.run(trace, realtime=realtime, keep=False, on_done=to_host)
    st = srv.dev.stats()
    srv.close()
    assert srv.peak_bytes <= budget and st["peak_outstanding"] <= budget
    assert all(r.done_at is not None and r.latency >= 0 and r.released for r in reqs)
    for r in reqs:
        want = oracle.bfs_multi(graphs[r.graph], r.sources)
        np.testing.assert_array_equal(r.host, want, err_msg=f"request {r.rid} ({r.graph}, k={r.k})")
        assert r.depth == int(want.max()) + 1
    # requests shared the device: some request was admitted while another ran
    assert overlapping_pairs(reqs) > 0
    # the same requests alone give the same levels
    for r in reqs[:12]:
        h = handles[r.graph]
        alone = h.bfs_multi(r.sources) if r.k > 1 else h.bfs(int(r.sources[0])).view(1, -1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(alone.cpu().numpy(), r.host)
    s = summarize(reqs)
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_short_requests_overtake_a_long_one(resident):
    """A request on a 256 x 256 grid (hundreds of levels) is running when R-MAT
    requests arrive: they join the running sweep and finish many iterations before
    it does."""
    graphs, handles = resident
    grid = inputs.grid_workload(256, 0.9, seed=6, permute_seed=7)
    gh = blest.Graph(grid, reorder="bandwidth")
    g_src = inputs.sources(grid, seed=1, k=2)
    r_src = [inputs.sources(graphs["rmat"], seed=10 + i, k=3) for i in range(4)]
    trace = [(0.0, "grid", g_src)] + [(0.001 * (i + 1), "rmat", s) for i, s in enumerate(r_src)]
    srv = Server({"grid": gh, "rmat": handles["rmat"]}, 64 << 20)
    reqs = srv.run(trace, realtime=True, keep=False, on_done=to_host)
    srv.close()
    long = reqs[0]
    np.testing.assert_array_equal(long.host, oracle.bfs_multi(grid, g_src))
    print(f"grid request: iterations {long.admit_iter}..{long.done_iter}; rmat: " +
          ", ".join(f"{r.admit_iter}..{r.done_iter}" for r in reqs[1:]), flush=True)
    for r in reqs[1:]:
        np.testing.assert_array_equal(r.host, oracle.bfs_multi(graphs["rmat"], r.sources))
    joined = [r for r in reqs[1:] if long.admit_iter < r.admit_iter < long.done_iter]
    assert joined, "no request joined the running sweep"
    assert all(r.done_iter < long.done_iter for r in joined)
    gh.close()


def test_budget_bounds_device_memory_and_requests_queue(resident):
    graphs, handles = resident
    n_max = max(h.n for h in handles.values())
    budget = 4 * 64 * n_max            # one full-width request of the largest graph at a time
    trace = poisson_trace(9, 1e6, 40, list(graphs), src_of(graphs), k_max=64)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    srv = Server(handles, budget)
    reqs = srv.run(trace, realtime=False, keep=False, on_done=to_host)
    srv.close()
    assert srv.peak_bytes <= budget
    # outputs come from PyTorch's pool only once admitted: its peak stays in budget
    # (plus the copies' rounding)
    assert torch.cuda.max_memory_allocated() - base <= budget + 64 * 512
    for r in reqs:
        np.testing.assert_array_equal(r.host, oracle.bfs_multi(graphs[r.graph], r.sources))


def test_idle_launch_ends_and_restarts(resident):
    graphs, handles = resident
    import time
    srv = Server(handles, 64 << 20, idle_ms=5)
    iters = 0
    for round_ in range(3):
        s = inputs.sources(graphs["small"], seed=round_, k=5)
        reqs = srv.run([(0.0, "small", s)], keep=False, on_done=to_host)
        np.testing.assert_array_equal(reqs[0].host, oracle.bfs_multi(graphs["small"], s))
        iters += reqs[0].done_iter - reqs[0].admit_iter + 1
        time.sleep(0.05)  # the launch ends after 5 ms without work
        st = srv.dev.stats()
        assert not st["running"]
        # the phase totals are published when a launch ends: every iteration that
        # ran a request is counted, and every phase took some time
        assert st["iterations"] >= iters
        assert min(st["control_us"], st["stage1_us"], st["stage2_us"], st["admit_us"]) > 0
    assert srv.dev.stats()["launches"] >= 3
    srv.close()
    # ordinary calls run again after the server's launches ended
    s = int(inputs.sources(graphs["rmat"], seed=2, k=1)[0])
    np.testing.assert_array_equal(handles["rmat"].bfs(s).cpu().numpy(), oracle.bfs(graphs["rmat"], s))
