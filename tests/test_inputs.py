"""Checks of the shared seeded input generators (``inputs``): determinism, CSR
normal form, and the statistics each workload recipe is meant to have."""
from __future__ import annotations

import hashlib

import numpy as np

import inputs


def digest(g):
    h = hashlib.sha256()
    h.update(g.row_ptr.tobytes())
    h.update(g.col.tobytes())
    return h.hexdigest()


def assert_normal_form(g, symmetric=True):
    rp = g.row_ptr.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(g.col)
    tail = np.repeat(np.arange(g.n), np.diff(rp))
    head = g.col.astype(np.int64)
    assert np.all(head < g.n)
    assert not np.any(tail == head), "self-loop"
    key = tail * g.n + head
    assert np.all(np.diff(key) > 0), "rows not sorted or duplicate arcs"
    if symmetric:
        rkey = np.sort(head * g.n + tail)
        np.testing.assert_array_equal(rkey, key)


def test_rmat_deterministic_and_normal():
    a = inputs.rmat(12, 16, seed=5)
    b = inputs.rmat(12, 16, seed=5)
    c = inputs.rmat(12, 16, seed=6)
    assert digest(a) == digest(b) != digest(c)
    assert_normal_form(a)


def test_rmat_is_skewed():
    g = inputs.rmat(14, 16, seed=1)
    deg = np.sort(g.degrees())[::-1]
    assert deg[: g.n // 100].sum() > 0.05 * deg.sum()
    assert (deg == 0).sum() > 0.1 * g.n          # R-MAT leaves many vertices isolated


def test_grid_edges_and_bounds():
    g = inputs.grid(100, 80, 0.9, seed=2)
    assert_normal_form(g)
    full = 2 * (99 * 80 + 100 * 79)
    assert abs(g.nnz - 0.9 * full) < 0.02 * full
    deg = g.degrees()
    assert deg.max() <= 4
    full_grid = inputs.grid(7, 9, 1.0, seed=0)
    assert full_grid.nnz == 2 * (6 * 9 + 7 * 8)


def test_permutation_and_relabel():
    p = inputs.permutation(1000, 9)
    assert sorted(p.tolist()) == list(range(1000))
    assert not np.array_equal(p, np.arange(1000))
    g = inputs.rmat(10, 8, seed=1)
    h = inputs.relabel(g, p[: g.n] if g.n == 1000 else inputs.permutation(g.n, 9))
    assert_normal_form(h)
    assert h.nnz == g.nnz


def test_sources_have_degree_and_are_distinct_when_asked():
    g = inputs.rmat(12, 16, seed=3)
    s = inputs.sources(g, seed=4, k=64, distinct=True)
    assert len(s) == 64 and len(set(s.tolist())) == 64
    assert np.all(g.degrees()[s] > 0)
    np.testing.assert_array_equal(s, inputs.sources(g, seed=4, k=64, distinct=True))


def test_many_graphs_recipe_ranges():
    rec = inputs.many_graphs_recipe(256, base_seed=1000)
    scales = [r[0] for r in rec]
    efs = [r[1] for r in rec]
    assert min(scales) == 10 and max(scales) == 16
    assert min(efs) >= 8 and max(efs) <= 32
    assert len({r[2] for r in rec}) == 256


def test_from_arcs_normalises():
    g = inputs.from_arcs(5, [0, 0, 1, 2, 3, 3], [1, 1, 1, 3, 0, 0], False)
    assert_normal_form(g, symmetric=False)
    assert g.col.tolist() == [1, 3, 0] and g.row_ptr.tolist() == [0, 1, 1, 2, 3, 3]
