"""Pins for the BFS oracle (``oracle.bfs``): closed forms, exhaustive brute force on
tiny graphs, a library routine on mid-size graphs, invariants, and mutation tests
showing that plausible mistakes in the oracle fail these pins.

The oracle computes the level/parent arrays of the paper's problem statement
(Section 2): level[u] = length of a shortest source-to-u path along out-edges."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import inputs
import oracle
from tests import families


# ---------------------------------------------------------------------------
# Independent references used only by the pins
# ---------------------------------------------------------------------------

def dense_boolean_levels(adj: np.ndarray, s: int) -> np.ndarray:
    """Levels by repeated dense Boolean products R <- R or (A x R), with A the
    adjacency of the transposed graph (the pull form of Section 2)."""
    n = adj.shape[0]
    A = adj.T.astype(np.int64)
    reached = np.zeros(n, bool)
    reached[s] = True
    level = np.full(n, -1, np.int32)
    level[s] = 0
    ell = 0
    while True:
        ell += 1
        y = (A @ reached.astype(np.int64)) > 0
        new = y & ~reached
        if not new.any():
            return level
        level[new] = ell
        reached |= new


def floyd_warshall_levels(adj: np.ndarray) -> np.ndarray:
    n = adj.shape[0]
    INF = 10 ** 6
    d = np.where(adj > 0, 1, INF).astype(np.int64)
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, [k]] + d[[k], :])
    return np.where(d >= INF, -1, d).astype(np.int32)


def scipy_levels(g, s):
    m = sp.csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(g.n, g.n))
    d = shortest_path(m, directed=True, unweighted=True, indices=[s])[0]
    return np.where(np.isinf(d), -1, d).astype(np.int32)


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", sorted(families.ALL_FAMILIES))
def test_closed_forms_every_source(name):
    g, lv = families.ALL_FAMILIES[name]()
    for s in range(g.n):
        np.testing.assert_array_equal(oracle.bfs(g, s), lv(s), err_msg=f"{name} source {s}")


def test_single_vertex_graph():
    g = families.small_dense_csr(1, np.zeros((1, 1), np.uint8))
    np.testing.assert_array_equal(oracle.bfs(g, 0), [0])


def test_source_out_of_range_rejected():
    g, _ = families.path(4)
    with pytest.raises(ValueError):
        oracle.bfs(g, 4)


# ---------------------------------------------------------------------------
# Exhaustive brute force
# ---------------------------------------------------------------------------

def test_all_undirected_graphs_on_5_vertices():
    count = 0
    for adj in families.all_undirected(5):
        g = families.small_dense_csr(5, adj)
        for s in range(5):
            np.testing.assert_array_equal(oracle.bfs(g, s), dense_boolean_levels(adj, s))
        count += 1
    assert count == 1024


def test_all_directed_graphs_on_4_vertices():
    count = 0
    for adj in families.all_directed(4):
        g = families.small_dense_csr(4, adj)
        ref = floyd_warshall_levels(adj)
        for s in range(4):
            np.testing.assert_array_equal(oracle.bfs(g, s), ref[s])
        count += 1
    assert count == 4096


def test_random_directed_graphs_up_to_64_vertices():
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(1, 65))
        adj = (rng.random((n, n)) < rng.uniform(0.01, 0.2)).astype(np.uint8)
        np.fill_diagonal(adj, 0)
        g = families.small_dense_csr(n, adj)
        ref = floyd_warshall_levels(adj)
        for s in range(n):
            np.testing.assert_array_equal(oracle.bfs(g, s), ref[s])


# ---------------------------------------------------------------------------
# Library routine at mid size
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("graph", ["rmat12", "grid64"])
def test_matches_scipy_shortest_path(graph):
    g = inputs.rmat(12, 16, seed=11) if graph == "rmat12" else inputs.grid(64, 64, 0.9, seed=4)
    for s in inputs.sources(g, seed=2, k=4):
        np.testing.assert_array_equal(oracle.bfs(g, int(s)), scipy_levels(g, int(s)))


# ---------------------------------------------------------------------------
# Invariants at any size
# ---------------------------------------------------------------------------

def check_invariants(g, s, level):
    assert level[s] == 0
    deg = np.diff(g.row_ptr.astype(np.int64))
    tail = np.repeat(np.arange(g.n), deg)
    head = g.col.astype(np.int64)
    lt, lh = level[tail], level[head]
    both = (lt >= 0) & (lh >= 0)
    assert np.all(np.abs(lt[both] - lh[both]) <= 1)          # symmetric graphs
    assert np.all(lh[lt >= 0] >= 0)                          # reached closed under arcs
    # every vertex at level l > 0 has a neighbour at l - 1
    has_parent = np.zeros(g.n, bool)
    ok = (lt >= 0) & (lh == lt + 1)
    has_parent[head[ok]] = True
    reached = level > 0
    assert np.all(has_parent[reached])
    # reached set = the connected component of s
    m = sp.csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
                      shape=(g.n, g.n))
    _, lab = connected_components(m, directed=False)
    np.testing.assert_array_equal(level >= 0, lab == lab[s])


def test_invariants_rmat_and_grid():
    for g in (inputs.rmat_workload(14, 16, seed=3, permute_seed=9), inputs.grid(128, 96, 0.9, seed=6)):
        for s in inputs.sources(g, seed=1, k=3):
            check_invariants(g, int(s), oracle.bfs(g, int(s)))


def test_relabel_invariance():
    g = inputs.rmat(12, 8, seed=21)
    perm = inputs.permutation(g.n, 77)
    h = inputs.relabel(g, perm)
    for s in inputs.sources(g, seed=3, k=3):
        lg = oracle.bfs(g, int(s))
        lh = oracle.bfs(h, int(perm[s]))
        np.testing.assert_array_equal(lh[perm], lg)


# ---------------------------------------------------------------------------
# Parents (Graph500-style validation) and multi-source
# ---------------------------------------------------------------------------

def test_oracle_parents_are_valid_trees():
    g = inputs.rmat(12, 16, seed=8)
    for s in inputs.sources(g, seed=5, k=4):
        level, parent = oracle.bfs(g, int(s), parents=True)
        assert oracle.validate_tree(g, int(s), level, parent) == 0


def test_validator_catches_planted_parent_mistakes():
    g, _ = families.full_grid(6, 6)
    s = 14
    level, parent = oracle.bfs(g, s, parents=True)
    bad = parent.copy(); bad[s] = 0
    assert oracle.validate_tree(g, s, level, bad) == 1
    v = int(np.flatnonzero(level == 3)[0])
    bad = parent.copy(); bad[v] = s  # the source is three hops away: no arc s -> v
    assert oracle.validate_tree(g, s, level, bad) == 2
    bad = parent.copy(); bad[v] = v  # self-parent: no arc v->v
    assert oracle.validate_tree(g, s, level, bad) == 2
    # a neighbour on the same level (arc exists, level wrong)
    same = [int(w) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if level[w] == level[v]]
    nxt = [int(w) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if level[w] == level[v] + 1]
    if same or nxt:
        bad = parent.copy(); bad[v] = (same or nxt)[0]
        assert oracle.validate_tree(g, s, level, bad) == 3
    bad = parent.copy(); bad[v] = -1
    assert oracle.validate_tree(g, s, level, bad) == 4


def test_multi_is_loop_of_single_and_duplicates_agree():
    g = inputs.rmat(11, 16, seed=4)
    src = np.concatenate([inputs.sources(g, seed=9, k=5), inputs.sources(g, seed=9, k=2)])
    rows = oracle.bfs_multi(g, src)
    for j, s in enumerate(src):
        np.testing.assert_array_equal(rows[j], oracle.bfs(g, int(s)))
    np.testing.assert_array_equal(rows[0], rows[5])


# ---------------------------------------------------------------------------
# Mutation tests: a plausible mistake planted in a copy of the oracle must fail
# the pins above.  The copy is compiled into a temporary directory.
# ---------------------------------------------------------------------------

MUTANTS = {
    "step_two": ("level[w] = level[v] + 1;", "level[w] = level[v] + 2;"),
    "skip_last_neighbour": ("i < row_ptr[v + 1]; ++i) {\n      uint32_t w", "i + 1 < row_ptr[v + 1]; ++i) {\n      uint32_t w"),
    "source_level_one": ("level[source] = 0;", "level[source] = 1;"),
    "lifo_not_fifo": ("uint32_t v = queue[head++];", "uint32_t v = queue[--tail]; head = head;"),
}


def _pins_pass(bfs):
    for name in ("path17", "star9", "grid5x7", "k3_5"):
        g, lv = families.ALL_FAMILIES[name]()
        for s in range(g.n):
            if not np.array_equal(bfs(g, s), lv(s)):
                return False
    for adj in list(families.all_directed(3)):
        g = families.small_dense_csr(3, adj)
        ref = floyd_warshall_levels(adj)
        for s in range(3):
            if not np.array_equal(bfs(g, s), ref[s]):
                return False
    return True


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_fails_pins(mutant, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "bfs_oracle.c")).read()
    old, new = MUTANTS[mutant]
    assert old in src, "mutation anchor missing from the oracle source"
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / "mut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    p32 = ctypes.POINTER(ctypes.c_uint32)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_bfs.argtypes = [ctypes.c_uint32, p32, p32, ctypes.c_uint32, pi32, pi32]

    def mut_bfs(g, s):
        rp = np.ascontiguousarray(g.row_ptr, np.uint32)
        col = np.ascontiguousarray(g.col if len(g.col) else np.zeros(1, np.uint32), np.uint32)
        out = np.empty(g.n, np.int32)
        lib.oracle_bfs(g.n, rp.ctypes.data_as(p32), col.ctypes.data_as(p32), s, out.ctypes.data_as(pi32), None)
        return out

    assert _pins_pass(oracle.bfs)
    assert not _pins_pass(mut_bfs), f"mutant {mutant} slipped through the pins"
