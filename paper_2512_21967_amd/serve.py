"""Serving loop: BFS queries against device-resident graphs with continuous
batching on the device.

A request names a resident graph and 1..64 sources.  The device side is libblest's
server (``blest_server_*``): one persistent launch that keeps 64 source columns
per resident graph and, at every level boundary, admits waiting requests into
free columns, so a request that arrives while others run joins the running
sweep; its columns advance one level per server iteration alongside the others'
and are freed when they stop growing.  Each request's rows are the k-source BFS
of its sources (Section 2's stacked frontiers), identical to the request run
alone.

This host loop only moves requests from the trace into the server: oldest first,
each as soon as its output (k * n * 4 bytes, allocated from PyTorch's pool when the
request is submitted) fits the HBM budget together with the outputs of submitted
requests that have not been released.  A finished request's output stays charged
until the caller releases it (``keep=True``) or until ``on_done`` has consumed it
(``keep=False``: released right after ``on_done`` returns).

Latency is measured from a request's arrival to the moment the host sees it done
(its levels are then complete in device memory).
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    graph: str
    sources: np.ndarray            # uint32[k]
    arrival: float                 # host seconds (perf_counter base)
    levels: object = None          # int32 CUDA tensor [k, n] once submitted
    submitted_at: float | None = None
    done_at: float | None = None
    ticket: int | None = None
    depth: int = 0                 # 1 + deepest level over the request's rows
    admit_iter: int = 0            # server iteration that admitted it
    done_iter: int = 0             # server iteration after which it finished
    released: bool = False

    @property
    def k(self) -> int:
        return int(self.sources.size)

    @property
    def latency(self) -> float | None:
        return None if self.done_at is None else self.done_at - self.arrival


def poisson_trace(seed: int, rate_per_s: float, count: int, graphs, sources_of, k_max: int = 64):
    """Seeded request trace: exponential inter-arrival times at `rate_per_s`, graph
    uniform over `graphs`, k = 1 with probability 1/2 else uniform on 1..k_max,
    sources drawn by sources_of(graph, seed, k)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        g = graphs[int(rng.integers(len(graphs)))]
        k = 1 if rng.random() < 0.5 else int(rng.integers(1, k_max + 1))
        out.append((t, g, np.asarray(sources_of(g, int(rng.integers(1 << 30)), k), np.uint32)))
    return out


class Server:
    """Feeds request traces to a device server over resident graphs
    (name -> paper_2512_21967_amd.Graph).  `device_server` may replace the libblest
    server by any object with submit/poll/release (host-side tests)."""

    def __init__(self, graphs: dict, hbm_budget: int, idle_ms: int = 20, device_server=None, alloc=None):
        self.graphs = graphs
        self.names = list(graphs)
        self.index = {name: i for i, name in enumerate(self.names)}
        self.budget = int(hbm_budget)
        for name, g in graphs.items():
            if self.footprint(name, 1) > self.budget:
                raise ValueError(f"graph {name}: one source's output needs more than the HBM budget")
        if device_server is None:
            from . import DeviceServer
            device_server = DeviceServer([graphs[n] for n in self.names], self.budget, idle_ms)
        self.dev = device_server
        self.alloc = alloc if alloc is not None else self._torch_alloc
        self.outstanding = 0
        self.peak_bytes = 0

    def _torch_alloc(self, k, n):
        import torch
        return torch.empty((k, n), dtype=torch.int32, device=torch.device("cuda", self.graphs[self.names[0]].device))

    def footprint(self, graph: str, k: int) -> int:
        """Output bytes a request of k sources holds until it is released."""
        return 4 * int(k) * int(self.graphs[graph].n)

    def release(self, r: Request):
        if r.released or r.ticket is None:
            return
        self.dev.release(r.ticket)
        self.outstanding -= self.footprint(r.graph, r.k)
        r.released = True

    def run(self, trace, realtime: bool = True, keep: bool = True, on_done=None, poll_sleep: float = 20e-6,
            progress=None, progress_s: float = 30.0):
        """Replays `trace` [(t_arrival, graph, sources)] and returns the requests.
        realtime=False makes every request arrive at t = 0 (a closed-loop stress
        test).  keep=False releases each request (and drops its output) right after
        on_done(request) returns.  progress(done, total), if given, is called about
        every progress_s seconds."""
        t0 = time.perf_counter()
        t_prog, n_done = t0, 0
        reqs = [Request(i, g, np.asarray(s, np.uint32), t0 + (t if realtime else 0.0)) for i, (t, g, s) in
                enumerate(trace)]
        arrivals = collections.deque(reqs)
        waiting = collections.deque()
        inflight = {}
        while arrivals or waiting or inflight:
            now = time.perf_counter()
            while arrivals and arrivals[0].arrival <= now:
                waiting.append(arrivals.popleft())
            progressed = False
            # oldest first; the head waits until its output fits the budget
            while waiting:
                r = waiting[0]
                nbytes = self.footprint(r.graph, r.k)
                if self.outstanding + nbytes > self.budget:
                    break
                # the output is referenced by the request only, so that releasing the
                # request frees it
                r.levels = self.alloc(r.k, self.graphs[r.graph].n)
                t = self.dev.submit(self.index[r.graph], r.sources, r.levels)
                if t is None:  # the device's ring is full: wait for releases
                    r.levels = None
                    break
                waiting.popleft()
                r.ticket, r.submitted_at = t, time.perf_counter()
                self.outstanding += nbytes
                self.peak_bytes = max(self.peak_bytes, self.outstanding)
                inflight[t] = r
                progressed = True
            for t in list(inflight):
                state, depth, a, d = self.dev.poll(t)
                if state != 2:
                    continue
                r = inflight.pop(t)
                r.done_at = time.perf_counter()
                n_done += 1
                r.depth, r.admit_iter, r.done_iter = depth, a, d
                progressed = True
                if on_done is not None:
                    on_done(r)
                if not keep:
                    self.release(r)
                    r.levels = None
            if keep and waiting and not inflight and not progressed and \
                    self.outstanding + self.footprint(waiting[0].graph, waiting[0].k) > self.budget:
                raise RuntimeError("budget held by kept requests: release them or use keep=False")
            if progress is not None and time.perf_counter() - t_prog > progress_s:
                t_prog = time.perf_counter()
                progress(n_done, len(reqs))
            if not progressed:
                time.sleep(poll_sleep)
        return reqs

    def close(self):
        if hasattr(self.dev, "close"):
            self.dev.close()


def overlapping_pairs(reqs) -> int:
    """Pairs of requests that were on the device at once: admitted before the
    other finished, in server iterations."""
    iv = sorted((r.admit_iter, r.done_iter) for r in reqs if r.done_at is not None)
    count = 0
    for i, (a, d) in enumerate(iv):
        for a2, d2 in iv[i + 1:]:
            if a2 >= d:
                break
            count += 1
    return count


def summarize(reqs, edges_of=None):
    """p50/p99 latency (ms) and, given edges_of(request) -> traversed edges,
    throughput in GTEPS over the trace's makespan."""
    lat = np.array([r.latency for r in reqs]) * 1000.0
    out = {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean())}
    if edges_of is not None:
        span = max(r.done_at for r in reqs) - min(r.arrival for r in reqs)
        out["gteps"] = float(sum(edges_of(r) for r in reqs) / span / 1e9)
    return out
