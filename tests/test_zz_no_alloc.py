"""The allocation-free single-source entry point (blest_bfs_noalloc), called through
the C-ABI: its levels equal blest_bfs's (integers, tolerance 0) and the oracle's on
two calls in a row, the second on a smaller graph, so the shared static scratch
holds the first call's larger state when the second starts; and a graph whose
per-call state exceeds the scratch is refused before anything is enqueued."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
blest = pytest.importorskip("paper_2512_21967_amd")


@pytest.mark.gpu
@pytest.mark.parametrize("update", ["lazy", "eager"])
def test_noalloc_matches_bfs_on_two_calls_second_smaller(update):
    big = inputs.rmat_workload(16, 16, seed=5, permute_seed=6)
    small = inputs.rmat_workload(11, 8, seed=7, permute_seed=8)
    gb = blest.Graph(big, update=update, reorder="compression", window=4096)
    gs = blest.Graph(small, update=update, reorder="none")
    for gr, g in ((big, gb), (small, gs)):
        s = int(inputs.sources(gr, seed=9, k=1)[0])
        print(f"noalloc {update}: n={gr.n} source {s}", flush=True)
        out = torch.full((gr.n,), 123, dtype=torch.int32, device="cuda")
        g.bfs_noalloc(s, out)
        ref = g.bfs(s)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got, ref.cpu().numpy())
        np.testing.assert_array_equal(got, oracle.bfs(gr, s))
    gb.close()
    gs.close()


@pytest.mark.gpu
def test_noalloc_repeated_and_across_streams():
    gr = inputs.grid_workload(64, 0.9, seed=1, permute_seed=2)
    g = blest.Graph(gr, reorder="bandwidth")
    srcs = [int(x) for x in inputs.sources(gr, seed=3, k=4)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for _ in srcs]
    for i, s in enumerate(srcs):
        with torch.cuda.stream(streams[i % 2]):
            g.bfs_noalloc(s, outs[i], stream=streams[i % 2])
    torch.cuda.synchronize()
    for s, o in zip(srcs, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), oracle.bfs(gr, s))
    g.close()


def test_noalloc_refuses_state_beyond_scratch():
    """n = 2^26 vertices need 64 MiB of reached bytes alone: more than the scratch."""
    n = 1 << 26
    gr = inputs.from_arcs(n, [0, 1], [1, 2], True)
    g = blest.Graph(gr, reorder="none", device=-1)
    out = ctypes.c_void_p(1 << 20)  # never dereferenced: the size check comes first
    rc = blest.lib().blest_bfs_noalloc(g.handle, 0, out, None)
    assert rc == 5  # BLEST_ERR_BUDGET
    small = blest.Graph(inputs.rmat(8, 4, seed=1), reorder="none", device=-1)
    assert blest.lib().blest_bfs_noalloc(small.handle, 0, out, None) == 7  # host-only: no device
    assert blest.lib().blest_bfs_noalloc(small.handle, 1 << 20, out, None) == 1  # source >= n
