"""Autotuner: candidate enumeration, the per-class store of choices and its lookup
(CPU), and tuning runs whose winner must reproduce the oracle's levels (GPU)."""
import os

import numpy as np
import pytest

import inputs
import oracle
from paper_2512_21967_amd import autotune
from tests import families


def test_candidates_respect_the_register_cap():
    c = autotune.candidates()
    assert all(sl * gr <= 16 for _, sl, gr, _, _ in c)
    assert (8, 2, 2, "lazy", 0) in c and (8, 8, 4, "eager", 0) not in c
    assert {sg for sg, *_ in c} == {8, 16, 32} and {up for _, _, _, up, _ in c} == {"eager", "lazy", "adaptive"}
    assert autotune.candidates(sigmas=(8,), slots=(4,), groups=(4,), max_slots_in_flight=8) == []
    # thresholds multiply the adaptive candidates only
    c = autotune.candidates((8,), (2,), (2,), ("lazy", "adaptive"), (0, 64, 4096))
    assert c == [(8, 2, 2, "lazy", 0), (8, 2, 2, "adaptive", 0), (8, 2, 2, "adaptive", 64),
                 (8, 2, 2, "adaptive", 4096)]


def test_graph_key_classes_and_sizes():
    assert autotune.graph_key(inputs.rmat(12, 16, seed=1)) == "skewed-s12-k1"
    assert autotune.graph_key(inputs.grid(64, 64, 0.9, seed=1), k=64) == "mesh-s12-kmulti"
    star, _ = families.star(1000)
    assert autotune.graph_key(star).startswith("skewed-s10")
    path, _ = families.path(3000)
    assert autotune.graph_key(path) == "mesh-s12-k1"


def test_store_and_lookup_round_trip(tmp_path):
    p = os.path.join(tmp_path, "tuned.json")
    gr = inputs.rmat(11, 8, seed=2)
    assert autotune.lookup(gr, path=p) == ("skewed-s11-k1", None)
    best = autotune.Trial(8, 4, 1, "adaptive", 1.5, 4096)
    other = autotune.Trial(16, 2, 2, "lazy", 2.5)
    autotune.save("skewed-s11-k1", best, [other, best], "unit", path=p)
    key, opts = autotune.lookup(gr, path=p)
    assert key == "skewed-s11-k1"
    assert opts == {"sigma": 8, "slots": 4, "group": 1, "update": "adaptive", "eager_max": 4096}
    db = autotune.load(p)
    assert [c["ms"] for c in db[key]["candidates"]] == [1.5, 2.5]
    # a second class is added beside the first
    autotune.save("mesh-s12-k1", other, [other], "unit", path=p)
    assert set(autotune.load(p)) == {"skewed-s11-k1", "mesh-s12-k1"}


def test_grid_cap_is_stored_only_when_set(tmp_path):
    p = os.path.join(tmp_path, "tuned.json")
    gr = inputs.grid(64, 64, 0.9, seed=1)
    capped = autotune.Trial(8, 1, 1, "eager", 3.0, 0, 64)
    full = autotune.Trial(8, 1, 1, "eager", 4.0)
    assert capped.options()["max_grid"] == 64 and "max_grid" not in full.options()
    autotune.save(autotune.graph_key(gr), capped, [full, capped], "unit", path=p)
    _, opts = autotune.lookup(gr, path=p)
    assert opts["max_grid"] == 64
    assert [c.get("max_grid", 0) for c in autotune.load(p)[autotune.graph_key(gr)]["candidates"]] == [64, 0]


def test_committed_choices_are_valid_options():
    for key, rec in autotune.load().items():
        o = rec["options"]
        assert o["sigma"] in (8, 16, 32) and o["slots"] in (1, 2, 4, 8) and o["group"] in (1, 2, 4)
        assert o["update"] in ("eager", "lazy", "adaptive") and o["eager_max"] >= 0
        assert o.get("max_grid", 0) >= 0
        assert rec["candidates"][0]["ms"] == rec["ms"]


@pytest.mark.gpu
@pytest.mark.parametrize("k", [1, 8])
def test_autotune_winner_reproduces_the_oracle(k):
    import paper_2512_21967_amd as blest
    gr = inputs.rmat_workload(12, 16, seed=4, permute_seed=5)
    srcs = inputs.sources(gr, seed=6, k=max(k, 2), distinct=True)
    cands = [(8, 1, 1, "eager", 0), (8, 2, 2, "lazy", 0), (8, 2, 2, "adaptive", 16), (16, 4, 2, "lazy", 0),
             (32, 2, 4, "eager", 0)]
    best, trials = autotune.autotune(gr, srcs, k=k, cands=cands, repeats=2)
    assert best in trials and all(t.ms > 0 for t in trials)
    assert len(trials) == (5 if k == 1 else 4)
    g = blest.Graph(gr, **best.options())
    if k == 1:
        for s in srcs:
            np.testing.assert_array_equal(g.bfs(int(s)).cpu().numpy(), oracle.bfs(gr, int(s)))
    else:
        got = g.bfs_multi(srcs[:k]).cpu().numpy()
        for j, s in enumerate(srcs[:k]):
            np.testing.assert_array_equal(got[j], oracle.bfs(gr, int(s)))
