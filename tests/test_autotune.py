"""Autotuner: candidate enumeration (CPU) and a tuning run whose winner must
reproduce the oracle's levels (GPU)."""
import numpy as np
import pytest

import inputs
import oracle
from paper_2512_21967_amd import autotune


def test_candidates_respect_the_register_cap():
    c = autotune.candidates()
    assert all(sl * gr <= 16 for _, sl, gr, _ in c)
    assert (8, 2, 2, "lazy") in c and (8, 8, 4, "eager") not in c
    assert {sg for sg, *_ in c} == {8, 16, 32} and {up for *_, up in c} == {"eager", "lazy"}
    assert autotune.candidates(sigmas=(8,), slots=(4,), groups=(4,), max_slots_in_flight=8) == []


@pytest.mark.gpu
@pytest.mark.parametrize("k", [1, 8])
def test_autotune_winner_reproduces_the_oracle(k):
    import paper_2512_21967_amd as blest
    gr = inputs.rmat_workload(12, 16, seed=4, permute_seed=5)
    srcs = inputs.sources(gr, seed=6, k=max(k, 2), distinct=True)
    cands = [(8, 1, 1, "eager"), (8, 2, 2, "lazy"), (16, 4, 2, "lazy"), (32, 2, 4, "eager")]
    best, trials = autotune.autotune(gr, srcs, k=k, cands=cands, repeats=2)
    assert best in trials and all(t.ms > 0 for t in trials)
    assert len(trials) == 4
    g = blest.Graph(gr, **best.options())
    if k == 1:
        for s in srcs:
            np.testing.assert_array_equal(g.bfs(int(s)).cpu().numpy(), oracle.bfs(gr, int(s)))
    else:
        got = g.bfs_multi(srcs[:k]).cpu().numpy()
        for j, s in enumerate(srcs[:k]):
            np.testing.assert_array_equal(got[j], oracle.bfs(gr, int(s)))
