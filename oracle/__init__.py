"""Oracle for the BLEST hot path (Elbek and Kaya, BLEST: Blazingly Efficient BFS using
Tensor Cores).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The GPU library never
calls it and shares no code with it; the only inputs both sides share come from the
seeded generators in ``inputs/``.

Contents
  * ``bfs``/``bfs_multi``/``validate_tree`` - plain FIFO-queue BFS in C
    (``bfs_oracle.c``): the definition of the level and parent arrays of the paper's
    problem statement (Section 2).  Multi-source is a loop of single-source runs
    (stacking frontiers column-wise, Section 2, does not change any column).
  * ``oracle.bvss`` - slices by their definition (Section 2), the virtual-slice-set
    rules (Section 2.1), column-major placement (Section 2.1.2), compression ratio
    and update divergence (Sections 2.2 and 2.2.1), and the Table 3 byte accounting.
  * ``oracle.reorder`` - JaccardWithWindows (Algorithm 1) step by step, the
    social-like test (Section 2.2.1) and reverse Cuthill-McKee with the tie rules
    listed in its docstring.
  * ``oracle.prepass`` - the shingle ordering (min-hashes of out-neighbour sets,
    SplitMix64 hash functions) that stands in for Gorder before Algorithm 1
    (Section 2.2), and its composition with Algorithm 1.

Graphs are duck-typed: any object with ``n``, ``row_ptr`` (uint32[n+1]) and ``col``
(uint32[nnz]) holding sorted out-neighbour lists.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compiles bfs_oracle.c (plain C, -O2, single-threaded) into liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                               os.path.join(_HERE, "bfs_oracle.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    u32 = ctypes.c_uint32
    p32 = ctypes.POINTER(ctypes.c_uint32)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_bfs.restype = ctypes.c_int
    lib.oracle_bfs.argtypes = [u32, p32, p32, u32, pi32, pi32]
    lib.oracle_bfs_multi.restype = ctypes.c_int
    lib.oracle_bfs_multi.argtypes = [u32, p32, p32, p32, u32, pi32]
    lib.oracle_validate_tree.restype = ctypes.c_int
    lib.oracle_validate_tree.argtypes = [u32, p32, p32, u32, pi32, pi32]
    _lib = lib
    return lib


def _u32p(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _i32p(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _graph_ptrs(g):
    rp, prp = _u32p(g.row_ptr)
    col = g.col if len(g.col) else np.zeros(1, np.uint32)
    col, pcol = _u32p(col)
    return (rp, col), prp, pcol


def bfs(g, source: int, parents: bool = False):
    """Levels (int32[n], -1 = unreachable) from `source`; with parents=True also the
    FIFO-discovery parent array."""
    keep, prp, pcol = _graph_ptrs(g)
    level = np.empty(g.n, dtype=np.int32)
    parent = np.empty(g.n, dtype=np.int32) if parents else None
    rc = _load().oracle_bfs(g.n, prp, pcol, int(source), _i32p(level),
                            _i32p(parent) if parents else None)
    if rc != 0:
        raise ValueError(f"oracle_bfs failed for source {source} (n={g.n})")
    return (level, parent) if parents else level


def bfs_multi(g, sources) -> np.ndarray:
    """int32[k, n]; row j is the BFS from sources[j]."""
    keep, prp, pcol = _graph_ptrs(g)
    src, psrc = _u32p(sources)
    out = np.empty((len(src), g.n), dtype=np.int32)
    rc = _load().oracle_bfs_multi(g.n, prp, pcol, psrc, len(src), _i32p(out))
    if rc != 0:
        raise ValueError("oracle_bfs_multi failed")
    return out


def validate_tree(g, source: int, level: np.ndarray, parent: np.ndarray) -> int:
    """0 if `parent` is a valid BFS tree for the (trusted) `level`, else the number of
    the first Graph500-style rule broken (see bfs_oracle.c)."""
    keep, prp, pcol = _graph_ptrs(g)
    level = np.ascontiguousarray(level, dtype=np.int32)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    return int(_load().oracle_validate_tree(g.n, prp, pcol, int(source), _i32p(level), _i32p(parent)))
