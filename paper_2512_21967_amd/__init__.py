"""Python binding of libblest: pull-based BFS over Binarised Virtual Slice Sets on
MI355X (Elbek and Kaya, "BLEST: Blazingly Efficient BFS using Tensor Cores").

Argument marshalling only: every step of the BFS runs in the HIP kernels behind the
C-ABI declared in ``include/blest.h``.  PyTorch supplies device memory and streams.
There is no CPU fallback: if ``libblest.so`` is missing or the device call fails,
the call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblest.so")

BLEST_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "invalid graph", 3: "too large", 4: "out of memory",
          5: "budget", 6: "device error", 7: "no device", 8: "internal error"}
REORDER = {"auto": 0, "none": 1, "compression": 2, "bandwidth": 3}
PREPASS = {"auto": 0, "off": 1, "shingle": 2}
UPDATE = {"auto": 0, "eager": 1, "lazy": 2, "adaptive": 3}
HUBS = {"auto": 0, "off": 1, "on": 2}
LDS_OFF = 0xFFFFFFFF
EXPORT = {"new_id": (0, np.uint32), "real_ptrs": (1, np.uint32), "virtual_to_real": (2, np.uint32),
          "vss_begin": (3, np.uint32), "row_ids": (4, np.uint32), "masks": (5, np.uint8),
          "vss_range": (6, np.uint8), "order_id": (7, np.uint32),
          "prepass_id": (8, np.uint32)}
EXPORTED_SYMBOLS = ("blest_default_options", "blest_build", "blest_bfs", "blest_bfs_noalloc", "blest_bfs_multi",
                    "blest_bfs_many",
                    "blest_batch_create", "blest_batch_run", "blest_batch_destroy", "blest_server_create",
                    "blest_server_submit", "blest_server_poll", "blest_server_release", "blest_server_stats",
                    "blest_server_destroy", "blest_configure", "blest_stats", "blest_footprint", "blest_export",
                    "blest_model_bytes", "blest_level_stats", "blest_barrier_probe", "blest_shutdown",
                    "blest_destroy", "blest_status_string")


class ServerStats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_uint64), ("outstanding", ctypes.c_uint64), ("peak_outstanding", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("submitted", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("running", ctypes.c_int32), ("grid", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("iterations", ctypes.c_uint64), ("control_us", ctypes.c_double), ("stage1_us", ctypes.c_double),
                ("stage2_us", ctypes.c_double), ("admit_us", ctypes.c_double)]


class BlestError(RuntimeError):
    def __init__(self, call, status):
        self.status = status
        super().__init__(f"{call} failed: {STATUS.get(status, status)} ({status})")


class Options(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("reorder", ctypes.c_int32), ("update", ctypes.c_int32), ("device", ctypes.c_int32),
                ("threads", ctypes.c_uint32), ("block", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("group", ctypes.c_uint32), ("ranges", ctypes.c_uint32), ("hubs", ctypes.c_uint32),
                ("lds_kib", ctypes.c_uint32), ("eager_max", ctypes.c_uint32), ("pack", ctypes.c_uint32),
                ("multi_ranges", ctypes.c_uint32), ("prepass", ctypes.c_uint32), ("shingles", ctypes.c_uint32),
                ("shingle_seed", ctypes.c_uint64), ("max_grid", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m", ctypes.c_uint64), ("sigma", ctypes.c_uint32),
                ("tau", ctypes.c_uint32), ("lanes", ctypes.c_uint32), ("num_slice_sets", ctypes.c_uint32),
                ("num_vss", ctypes.c_uint32), ("num_slices", ctypes.c_uint64), ("compression", ctypes.c_double),
                ("u_div_paper", ctypes.c_double), ("u_div_native", ctypes.c_double),
                ("social_like", ctypes.c_int32), ("reorder_used", ctypes.c_int32), ("update_used", ctypes.c_int32),
                ("nranges", ctypes.c_uint32), ("range_len", ctypes.c_uint32),
                ("bvss_device_bytes", ctypes.c_uint64), ("bvss_bytes_table3", ctypes.c_uint64),
                ("reorder_seconds", ctypes.c_double), ("build_seconds", ctypes.c_double),
                ("hubs_sorted", ctypes.c_int32), ("lds_bytes", ctypes.c_uint32),
                ("lds_chunk_words", ctypes.c_uint32), ("hub_cpos", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("block", ctypes.c_uint32), ("kernel_vgprs", ctypes.c_uint32),
                ("blocks_per_cu_runtime", ctypes.c_uint32), ("blocks_per_cu_own", ctypes.c_uint32),
                ("eager_max", ctypes.c_uint32), ("packed", ctypes.c_int32), ("multi_ranges", ctypes.c_uint32),
                ("multi_num_vss", ctypes.c_uint32), ("prepass_used", ctypes.c_int32),
                ("prepass_seconds", ctypes.c_double), ("window_used", ctypes.c_uint32)]


_lib = None


def lib():
    """Loads libblest.so (building it only if it has never been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    # PyTorch ships its own HIP runtime under the same soname as the system one; it
    # has to be the one in the process (loaded first), or a later torch.cuda call
    # runs on the other copy and finds no GPU
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    p32 = ctypes.POINTER(ctypes.c_uint32)
    L.blest_default_options.argtypes = [ctypes.POINTER(Options)]
    L.blest_default_options.restype = None
    L.blest_build.argtypes = [u32, u64, p32, p32, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.blest_build.restype = ctypes.c_int
    L.blest_bfs.argtypes = [vp, u32, vp, vp, vp]
    L.blest_bfs.restype = ctypes.c_int
    L.blest_bfs_noalloc.argtypes = [vp, u32, vp, vp]
    L.blest_bfs_noalloc.restype = ctypes.c_int
    L.blest_bfs_multi.argtypes = [vp, p32, u32, vp, vp]
    L.blest_bfs_multi.restype = ctypes.c_int
    L.blest_bfs_many.argtypes = [ctypes.POINTER(vp), p32, u32, ctypes.POINTER(vp), vp]
    L.blest_bfs_many.restype = ctypes.c_int
    L.blest_batch_create.argtypes = [ctypes.POINTER(vp), p32, u32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.blest_batch_create.restype = ctypes.c_int
    L.blest_batch_run.argtypes = [vp, vp]
    L.blest_batch_run.restype = ctypes.c_int
    L.blest_batch_destroy.argtypes = [vp]
    L.blest_batch_destroy.restype = None
    L.blest_server_create.argtypes = [ctypes.POINTER(vp), u32, u64, u32, ctypes.POINTER(vp)]
    L.blest_server_create.restype = ctypes.c_int
    L.blest_server_submit.argtypes = [vp, u32, p32, u32, vp, ctypes.POINTER(u64)]
    L.blest_server_submit.restype = ctypes.c_int
    L.blest_server_poll.argtypes = [vp, u64, ctypes.POINTER(i32), p32, p32, p32]
    L.blest_server_poll.restype = ctypes.c_int
    L.blest_server_release.argtypes = [vp, u64]
    L.blest_server_release.restype = ctypes.c_int
    L.blest_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.blest_server_stats.restype = ctypes.c_int
    L.blest_server_destroy.argtypes = [vp, u32]
    L.blest_server_destroy.restype = ctypes.c_int
    L.blest_configure.argtypes = [vp, i32, u32, u32, u32, u32]
    L.blest_configure.restype = ctypes.c_int
    L.blest_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.blest_stats.restype = ctypes.c_int
    L.blest_footprint.argtypes = [vp, u32, ctypes.POINTER(u64)]
    L.blest_footprint.restype = ctypes.c_int
    L.blest_export.argtypes = [vp, i32, vp, u64, ctypes.POINTER(u64)]
    L.blest_export.restype = ctypes.c_int
    L.blest_model_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), u32, ctypes.POINTER(u64)]
    L.blest_model_bytes.restype = ctypes.c_int
    L.blest_level_stats.argtypes = [i32, vp, u32, u32, vp, vp, vp, vp, vp, vp]
    L.blest_level_stats.restype = ctypes.c_int
    L.blest_barrier_probe.argtypes = [i32, u32, u32, u32, ctypes.POINTER(ctypes.c_double)]
    L.blest_barrier_probe.restype = ctypes.c_int
    L.blest_shutdown.argtypes = []
    L.blest_shutdown.restype = None
    L.blest_destroy.argtypes = [vp]
    L.blest_destroy.restype = None
    L.blest_status_string.argtypes = [ctypes.c_int]
    L.blest_status_string.restype = ctypes.c_char_p
    _lib = L
    # the library's process-wide HIP objects go while the runtime is still up
    atexit.register(L.blest_shutdown)
    return L


def _check(call, rc):
    if rc != BLEST_OK:
        raise BlestError(call, rc)


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require_int32_cuda(t, numel, what):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous int32 CUDA tensor")
    if t.numel() != numel:
        raise ValueError(f"{what} must hold {numel} elements, got {t.numel()}")


def default_options() -> Options:
    o = Options()
    lib().blest_default_options(ctypes.byref(o))
    return o


class Graph:
    """A graph resident on one GPU as a reordered BVSS (the handle of blest_build).

    `csr` is any object with `n`, `row_ptr` (uint32[n+1]) and `col` (uint32[nnz]),
    listing out-neighbours.  device=-1 builds the host structure only (statistics
    and exports work; BFS calls raise)."""

    def __init__(self, csr, *, sigma=8, slots=2, window=0, reorder="auto", update="auto",
                 device=0, threads=0, block=0, blocks_per_cu=0, group=0, ranges=0, hubs="auto", lds_kib=0,
                 eager_max=0, pack=True, multi_ranges=0, prepass="auto", shingles=0, shingle_seed=None,
                 max_grid=0):
        o = default_options()
        o.sigma, o.slots, o.window = sigma, slots, window
        o.reorder, o.update = REORDER[reorder], UPDATE[update]
        o.device, o.threads, o.block, o.blocks_per_cu = device, threads, block, blocks_per_cu
        o.group, o.ranges, o.hubs = group, ranges, HUBS[hubs]
        o.lds_kib = LDS_OFF if lds_kib is None else lds_kib
        o.eager_max = eager_max
        o.pack = 0 if pack else 1
        o.multi_ranges = multi_ranges
        o.prepass, o.shingles = PREPASS[prepass], shingles
        if shingle_seed is not None:
            o.shingle_seed = shingle_seed
        o.max_grid = max_grid
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.uint32)
        col = np.ascontiguousarray(csr.col if len(csr.col) else np.zeros(1, np.uint32), dtype=np.uint32)
        h = ctypes.c_void_p()
        _check("blest_build", lib().blest_build(int(csr.n), int(rp[-1]), _p32(rp), _p32(col), ctypes.byref(o),
                                                ctypes.byref(h)))
        self._h = h
        self.n = int(csr.n)
        self.device = device

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().blest_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- BFS -----------------------------------------------------------------
    def bfs(self, source: int, levels=None, parents=None, stream=None):
        """Levels (int32 CUDA tensor [n], -1 = unreachable) from `source`; with
        parents=True (or a tensor) also the parent array.  Asynchronous on `stream`."""
        import torch
        dev = torch.device("cuda", self.device)
        if levels is None:
            levels = torch.empty(self.n, dtype=torch.int32, device=dev)
        _require_int32_cuda(levels, self.n, "levels")
        par = None
        if parents is True:
            par = torch.empty(self.n, dtype=torch.int32, device=dev)
        elif parents is not None and parents is not False:
            par = parents
            _require_int32_cuda(par, self.n, "parents")
        _check("blest_bfs", lib().blest_bfs(self.handle, int(source), ctypes.c_void_p(levels.data_ptr()),
                                            ctypes.c_void_p(par.data_ptr() if par is not None else 0),
                                            _stream_ptr(stream)))
        return (levels, par) if par is not None else levels

    def bfs_noalloc(self, source: int, levels, stream=None):
        """Levels from `source` into the caller's int32 CUDA tensor [n] through
        blest_bfs_noalloc, which allocates nothing (its state lives in the
        library's static device scratch).  Asynchronous on `stream`."""
        _require_int32_cuda(levels, self.n, "levels")
        _check("blest_bfs_noalloc", lib().blest_bfs_noalloc(self.handle, int(source),
                                                            ctypes.c_void_p(levels.data_ptr()), _stream_ptr(stream)))
        return levels

    def bfs_multi(self, sources, levels=None, stream=None):
        """Levels of k <= 64 sources in one launch: int32 CUDA tensor [k, n]."""
        import torch
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        k = int(src.size)
        if levels is None:
            levels = torch.empty((k, self.n), dtype=torch.int32, device=torch.device("cuda", self.device))
        _require_int32_cuda(levels, k * self.n, "levels")
        _check("blest_bfs_multi", lib().blest_bfs_multi(self.handle, _p32(src), k,
                                                        ctypes.c_void_p(levels.data_ptr()), _stream_ptr(stream)))
        return levels

    # -- multi-source analytics on the k-source BFS ----------------------------
    def source_stats(self, sources, stream=None) -> dict:
        """Reached count, level sum, eccentricity, smallest farthest vertex and
        closeness (reached - 1) / sum of every source, from k-source BFS calls of
        up to 64 sources each; numpy arrays."""
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        parts = []
        for i in range(0, src.size, 64):
            st = level_stats(self.bfs_multi(src[i:i + 64], stream=stream), stream=stream)
            parts.append({k: v.cpu().numpy() for k, v in st.items()})
        return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]} if parts else {}

    def closeness(self, sources, stream=None) -> np.ndarray:
        return self.source_stats(sources, stream)["closeness"]

    def diameter_bounds(self, sources, sweeps=2, undirected=True, stream=None):
        """(lower, upper, sweep_sources) for the largest finite distance D: each
        sweep is one k-source BFS; lower = the largest eccentricity seen, the next
        sweep starting from the distinct farthest vertices of this one (at most 64,
        in first-seen order); upper = 2 * min eccentricity over rows that reached
        every vertex (the graph is then connected), for undirected graphs, else
        None."""
        src = [int(s) for s in sources][:64]
        lower, upper, used = -1, None, []
        for _ in range(max(1, sweeps)):
            st = self.source_stats(src, stream)
            used.append(list(src))
            lower = max(lower, int(st["ecc"].max()))
            if undirected:
                full = st["reached"] == self.n
                if full.any():
                    u = 2 * int(st["ecc"][full].min())
                    upper = u if upper is None else min(upper, u)
            nxt = []
            for f in st["far"]:
                f = int(f)
                if f != 0xFFFFFFFF and f not in nxt:
                    nxt.append(f)
            src = nxt[:64]
        return lower, upper, used

    def configure(self, update="auto", block=0, blocks_per_cu=0, group=0, eager_max=0):
        """Changes launch settings (update scheme, workgroup shape, group depth,
        adaptive threshold) without rebuilding."""
        _check("blest_configure", lib().blest_configure(self.handle, UPDATE[update], block, blocks_per_cu, group,
                                                        eager_max))

    # -- host-side information -------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        _check("blest_stats", lib().blest_stats(self.handle, ctypes.byref(s)))
        d = {name: getattr(s, name) for name, _ in Stats._fields_}
        d["reorder_used"] = {v: k for k, v in REORDER.items()}[d["reorder_used"]]
        d["update_used"] = {v: k for k, v in UPDATE.items()}[d["update_used"]]
        return d

    def footprint(self, k: int) -> int:
        b = ctypes.c_uint64()
        _check("blest_footprint", lib().blest_footprint(self.handle, int(k), ctypes.byref(b)))
        return int(b.value)

    def export(self, which: str) -> np.ndarray:
        code, dt = EXPORT[which]
        size = ctypes.c_uint64()
        _check("blest_export", lib().blest_export(self.handle, code, None, 0, ctypes.byref(size)))
        out = np.empty(max(size.value, 1) // np.dtype(dt).itemsize, dtype=dt)
        _check("blest_export", lib().blest_export(self.handle, code, out.ctypes.data_as(ctypes.c_void_p),
                                                  size.value, ctypes.byref(size)))
        return out[: size.value // np.dtype(dt).itemsize]

    def model_bytes(self, levels) -> int:
        """Algorithmic bytes of the call that produced `levels` ([n] or [k, n])."""
        lv = np.ascontiguousarray(levels, dtype=np.int32)
        if lv.size % self.n != 0 or lv.size == 0:
            raise ValueError("levels must hold k * n entries")
        b = ctypes.c_uint64()
        _check("blest_model_bytes", lib().blest_model_bytes(self.handle,
                                                            lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                            lv.size // self.n, ctypes.byref(b)))
        return int(b.value)


def level_stats(levels, stream=None) -> dict:
    """Per-row statistics of an int32 CUDA level tensor [k, n] (or [n]) computed on
    the device (``blest_level_stats``): reached (int64), total (int64, sum of the
    finite levels), ecc (int32, -1 for an empty row), far (int64, smallest vertex at
    level ecc, 0xFFFFFFFF for an empty row) and closeness (float64), as CUDA tensors
    of k entries."""
    import torch
    if not isinstance(levels, torch.Tensor) or levels.dtype != torch.int32 or not levels.is_cuda \
            or not levels.is_contiguous():
        raise TypeError("levels must be a contiguous int32 CUDA tensor")
    lv = levels if levels.dim() == 2 else levels.view(1, -1)
    k, n = int(lv.shape[0]), int(lv.shape[1])
    dev = lv.device
    reached = torch.empty(k, dtype=torch.int64, device=dev)
    total = torch.empty(k, dtype=torch.int64, device=dev)
    ecc = torch.empty(k, dtype=torch.int32, device=dev)
    far = torch.empty(k, dtype=torch.int32, device=dev)
    close = torch.empty(k, dtype=torch.float64, device=dev)
    _check("blest_level_stats", lib().blest_level_stats(
        dev.index if dev.index is not None else torch.cuda.current_device(), ctypes.c_void_p(lv.data_ptr()), k, n,
        ctypes.c_void_p(reached.data_ptr()), ctypes.c_void_p(total.data_ptr()), ctypes.c_void_p(ecc.data_ptr()),
        ctypes.c_void_p(far.data_ptr()), ctypes.c_void_p(close.data_ptr()), _stream_ptr(stream)))
    return {"reached": reached, "total": total, "ecc": ecc, "far": far.to(torch.int64) & 0xFFFFFFFF,
            "closeness": close}


def barrier_seconds(device: int = 0, block: int = 1024, rounds: int = 2000, max_grid: int = 0) -> float:
    """Seconds per grid barrier of the persistent launches (blest_barrier_probe),
    over at most max_grid workgroups when max_grid > 0."""
    x = ctypes.c_double()
    _check("blest_barrier_probe", lib().blest_barrier_probe(int(device), int(block), int(max_grid), int(rounds),
                                                            ctypes.byref(x)))
    return float(x.value)


def bfs_many(graphs, sources, outs=None, stream=None):
    """One launch running BFS i on graphs[i] from sources[i]; returns the list of
    int32 CUDA level tensors."""
    import torch
    g = len(graphs)
    src = np.ascontiguousarray(sources, dtype=np.uint32)
    if src.size != g:
        raise ValueError("one source per graph")
    if outs is None:
        outs = [torch.empty(gr.n, dtype=torch.int32, device=torch.device("cuda", gr.device)) for gr in graphs]
    for gr, o in zip(graphs, outs):
        _require_int32_cuda(o, gr.n, "levels")
    hs = (ctypes.c_void_p * g)(*[gr.handle.value for gr in graphs])
    ptrs = (ctypes.c_void_p * g)(*[o.data_ptr() for o in outs])
    _check("blest_bfs_many", lib().blest_bfs_many(hs, _p32(src), g, ptrs, _stream_ptr(stream)))
    return outs


class Batch:
    """A reusable many-graphs launch (blest_batch_*): BFS i on graphs[i] from
    sources[i] into outs[i].  run() enqueues one ordinary launch, so it can be
    captured into a CUDA/HIP graph.  Graphs and outputs must outlive the batch."""

    def __init__(self, graphs, sources, outs=None):
        import torch
        g = len(graphs)
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        if src.size != g:
            raise ValueError("one source per graph")
        if outs is None:
            outs = [torch.empty(gr.n, dtype=torch.int32, device=torch.device("cuda", gr.device)) for gr in graphs]
        for gr, o in zip(graphs, outs):
            _require_int32_cuda(o, gr.n, "levels")
        self.graphs, self.outs = list(graphs), list(outs)
        hs = (ctypes.c_void_p * g)(*[gr.handle.value for gr in graphs])
        ptrs = (ctypes.c_void_p * g)(*[o.data_ptr() for o in outs])
        h = ctypes.c_void_p()
        _check("blest_batch_create", lib().blest_batch_create(hs, _p32(src), g, ptrs, ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check("blest_batch_run", lib().blest_batch_run(self._h, _stream_ptr(stream)))
        return self.outs

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().blest_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BLEST_ERR_BUDGET = 5


class DeviceServer:
    """The continuous-batching server of libblest (blest_server_*): one persistent
    launch on its own stream serving requests of 1..64 sources on up to 4 resident
    graphs, admitted into free source columns at level boundaries.  Argument
    marshalling only; the loop that feeds it is ``paper_2512_21967_amd.serve``."""

    WAITING, RUNNING, DONE = 0, 1, 2

    def __init__(self, graphs, budget_bytes: int, idle_ms: int = 20):
        self.graphs = list(graphs)
        hs = (ctypes.c_void_p * len(self.graphs))(*[g.handle.value for g in self.graphs])
        h = ctypes.c_void_p()
        _check("blest_server_create", lib().blest_server_create(hs, len(self.graphs), int(budget_bytes), int(idle_ms),
                                                                ctypes.byref(h)))
        self._h = h

    def submit(self, graph: int, sources, levels):
        """Ticket of the submitted request, or None when the budget or the request
        ring is full (nothing was submitted)."""
        src = np.ascontiguousarray(sources, dtype=np.uint32)
        _require_int32_cuda(levels, src.size * self.graphs[graph].n, "levels")
        t = ctypes.c_uint64()
        rc = lib().blest_server_submit(self._h, int(graph), _p32(src), int(src.size),
                                       ctypes.c_void_p(levels.data_ptr()), ctypes.byref(t))
        if rc == BLEST_ERR_BUDGET:
            return None
        _check("blest_server_submit", rc)
        return int(t.value)

    def poll(self, ticket: int):
        """(state, levels, admit_iter, done_iter); state WAITING, RUNNING or DONE."""
        st = ctypes.c_int32()
        lv, a, d = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check("blest_server_poll", lib().blest_server_poll(self._h, int(ticket), ctypes.byref(st), ctypes.byref(lv),
                                                            ctypes.byref(a), ctypes.byref(d)))
        return int(st.value), int(lv.value), int(a.value), int(d.value)

    def release(self, ticket: int):
        _check("blest_server_release", lib().blest_server_release(self._h, int(ticket)))

    def stats(self) -> dict:
        s = ServerStats()
        _check("blest_server_stats", lib().blest_server_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServerStats._fields_}

    def close(self, timeout_ms: int = 60000):
        if getattr(self, "_h", None) is not None:
            _check("blest_server_destroy", lib().blest_server_destroy(self._h, int(timeout_ms)))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
