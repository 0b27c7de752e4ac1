"""Seeded synthetic inputs (graphs and BFS sources) shared by the oracle, the tests
and the benchmark.

This module holds none of the BFS method's arithmetic: it draws graphs and sources
and normalises them into a CSR whose neighbour lists are sorted, with self-loops and
duplicate arcs removed.  The native part is ``graphgen.cpp`` (counter-based
splitmix64 draws, so every graph depends only on its seed).

Workload recipes follow the synthetic stand-ins for the paper's two graph classes
(skewed "social-like" graphs and mesh-like road graphs; Section 2.2.1, Table 2):
R-MAT with the Graph500 initiator (0.57, 0.19, 0.19, 0.05) and a 4-neighbour grid
whose edges survive with probability p.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    """Compiles graphgen.cpp into libgraphgen.so next to this file."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "graphgen.cpp")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u32, u64, i32, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
    p32 = ctypes.POINTER(ctypes.c_uint32)
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [i32, i32, dbl, dbl, dbl, u64]
    lib.gg_grid.restype = vp
    lib.gg_grid.argtypes = [u32, u32, dbl, u64]
    lib.gg_from_arcs.restype = vp
    lib.gg_from_arcs.argtypes = [u32, u64, p32, p32, i32]
    lib.gg_permutation.restype = None
    lib.gg_permutation.argtypes = [u32, u64, p32]
    lib.gg_relabel.restype = vp
    lib.gg_relabel.argtypes = [u32, p32, p32, p32]
    lib.gg_sources.restype = u32
    lib.gg_sources.argtypes = [u32, p32, u64, u32, i32, p32]
    lib.gg_draw.restype = u64
    lib.gg_draw.argtypes = [u64, u64, u64]
    lib.gg_n.restype = u32
    lib.gg_n.argtypes = [vp]
    lib.gg_nnz.restype = u64
    lib.gg_nnz.argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, p32, p32]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


@dataclass
class Csr:
    """Out-neighbour CSR with 32-bit offsets and column indices."""
    n: int
    row_ptr: np.ndarray  # uint32[n + 1]
    col: np.ndarray      # uint32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _take(h, name="") -> Csr:
    lib = _load()
    if not h:
        raise ValueError("graph generator rejected its arguments")
    try:
        n = lib.gg_n(h)
        nnz = lib.gg_nnz(h)
        rp = np.empty(n + 1, dtype=np.uint32)
        col = np.empty(max(nnz, 1), dtype=np.uint32)
        lib.gg_copy(h, _p32(rp), _p32(col))
    finally:
        lib.gg_free(h)
    return Csr(n, rp, col[:nnz], name)


def rmat(scale: int, ef: int, seed: int, abcd=RMAT_ABCD) -> Csr:
    a, b, c, _ = abcd
    return _take(_load().gg_rmat(scale, ef, a, b, c, seed), f"rmat-s{scale}-ef{ef}-seed{seed}")


def grid(rows: int, cols: int, p: float, seed: int) -> Csr:
    return _take(_load().gg_grid(rows, cols, p, seed), f"grid-{rows}x{cols}-p{p}-seed{seed}")


def from_arcs(n: int, src, dst, symmetrise: bool) -> Csr:
    s = np.ascontiguousarray(src, dtype=np.uint32)
    d = np.ascontiguousarray(dst, dtype=np.uint32)
    if s.size == 0:
        s = np.zeros(1, np.uint32)
        d = np.zeros(1, np.uint32)  # a single self-loop, dropped by the normaliser
        if n == 0:
            raise ValueError("n must be positive")
    return _take(_load().gg_from_arcs(n, s.size, _p32(s), _p32(d), int(symmetrise)))


def permutation(n: int, seed: int) -> np.ndarray:
    p = np.empty(n, dtype=np.uint32)
    _load().gg_permutation(n, seed, _p32(p))
    return p


def relabel(g: Csr, perm: np.ndarray) -> Csr:
    """Vertex v of g becomes perm[v]."""
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    out = _take(_load().gg_relabel(g.n, _p32(g.row_ptr), _p32(g.col), _p32(perm)))
    out.name = g.name + "-perm"
    return out


def sources(g: Csr, seed: int, k: int, distinct: bool = False) -> np.ndarray:
    out = np.empty(max(k, 1), dtype=np.uint32)
    got = _load().gg_sources(g.n, _p32(g.row_ptr), seed, k, int(distinct), _p32(out))
    return out[:got]


def draw(seed: int, tag: int, counter: int) -> int:
    return int(_load().gg_draw(seed, tag, counter))


# ---------------------------------------------------------------------------
# Workload recipes (sizes of the benchmark configurations)
# ---------------------------------------------------------------------------

def rmat_workload(scale: int, ef: int = 16, seed: int = 1, permute_seed: int | None = None) -> Csr:
    """R-MAT graph; with permute_seed its labels are shuffled by a seeded permutation."""
    g = rmat(scale, ef, seed)
    if permute_seed is not None:
        g = relabel(g, permutation(g.n, permute_seed))
        g.name = f"rmat-s{scale}-ef{ef}-seed{seed}-perm{permute_seed}"
    return g


def grid_workload(side: int, p: float = 0.9, seed: int = 3, permute_seed: int | None = None) -> Csr:
    g = grid(side, side, p, seed)
    if permute_seed is not None:
        g = relabel(g, permutation(g.n, permute_seed))
        g.name = f"grid-{side}x{side}-p{p}-seed{seed}-perm{permute_seed}"
    return g


def many_graphs_recipe(count: int = 256, base_seed: int = 1000, scale_range=(10, 16), ef_range=(8, 32)):
    """(scale, ef, seed) for each of `count` R-MAT graphs: scale and edge factor drawn
    uniformly from the inclusive ranges with counter-based draws."""
    out = []
    for i in range(count):
        z = draw(base_seed, 7, i)
        s_lo, s_hi = scale_range
        e_lo, e_hi = ef_range
        scale = s_lo + (z & 0xFFFFFFFF) % (s_hi - s_lo + 1)
        ef = e_lo + (z >> 32) % (e_hi - e_lo + 1)
        out.append((int(scale), int(ef), base_seed + i))
    return out
