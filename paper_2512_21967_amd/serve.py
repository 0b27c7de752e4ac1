"""Serving loop: BFS queries against device-resident graphs, admitted by HBM
footprint and batched dynamically.

A request names a resident graph and 1..64 sources.  Requests for the same graph
that are waiting when a launch slot frees up are packed, oldest first, into the
columns of one k-source BFS (k <= 64, ``blest_bfs_multi``; a lone single source
uses ``blest_bfs``), as long as the batch's device footprint
(``blest_footprint``: bitmaps, queues and k*n*4 bytes of levels) fits the free part
of the HBM budget.  Requests that arrive while batches run join the next batch
that has room: a slot and budget are released as soon as a batch's completion
event fires.  Batches are issued on a small pool of streams, so the host forms
and launches the next batch, and the device copies or reduces finished results,
while the current BFS runs.  Persistent BFS launches themselves run one at a time
on the device (libblest serialises them so that each one's workgroups are all
resident).

Latency is measured from a request's arrival to the moment its levels are ready
on the device (the completion event of its batch, mapped to the host clock).
Each request's levels are row views into its batch's output and are identical to
what the request would get alone: every column of a k-source BFS is independent.
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
    levels: object = None          # int32 CUDA tensor [k, n] once done
    done_at: float | None = None
    batch_id: int | None = None

    @property
    def k(self) -> int:
        return int(self.sources.size)

    @property
    def latency(self) -> float | None:
        return None if self.done_at is None else self.done_at - self.arrival


def plan_batch(pending, free_bytes: int, footprint, max_k: int = 64):
    """Chooses the next batch.

    pending: dict graph -> deque of waiting Requests (oldest first).
    footprint(graph, k) -> device bytes a k-source call on that graph needs.
    Picks the graph whose oldest waiting request arrived first, then packs that
    graph's requests in arrival order while the column count stays <= max_k and
    the footprint fits free_bytes.  Returns (graph, [requests]) or None when the
    oldest request does not fit yet (head-of-line order is kept, so no request
    starves)."""
    heads = [(q[0].arrival, name) for name, q in pending.items() if q]
    if not heads:
        return None
    _, name = min(heads)
    q = pending[name]
    take, k = [], 0
    for r in q:
        if k + r.k > max_k:
            break
        if footprint(name, k + r.k) > free_bytes:
            break
        take.append(r)
        k += r.k
    if not take:
        return None
    return name, take


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
    """Runs request traces against resident graphs (name -> paper_2512_21967_amd.Graph)."""

    def __init__(self, graphs: dict, hbm_budget: int, streams: int = 2, max_k: int = 64):
        import torch
        self.torch = torch
        self.graphs = graphs
        self.budget = int(hbm_budget)
        self.max_k = max_k
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        for name, g in graphs.items():
            if g.footprint(1) > self.budget:
                raise ValueError(f"graph {name}: a single source needs more than the HBM budget")

    def footprint(self, graph: str, k: int) -> int:
        return self.graphs[graph].footprint(k)

    def _launch(self, name, reqs, stream, batch_id):
        torch = self.torch
        g = self.graphs[name]
        src = np.concatenate([r.sources for r in reqs]).astype(np.uint32)
        with torch.cuda.stream(stream):
            if src.size == 1:
                out = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
                g.bfs(int(src[0]), levels=out.view(-1), stream=stream)
            else:
                out = torch.empty((src.size, g.n), dtype=torch.int32, device="cuda")
                g.bfs_multi(src, levels=out, stream=stream)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        row = 0
        for r in reqs:
            r.levels = out[row:row + r.k]
            r.batch_id = batch_id
            row += r.k
        return done

    def run(self, trace, realtime: bool = True):
        """Replays `trace` [(t_arrival, graph, sources)] and returns the requests.
        realtime=False submits everything at t = 0 (a closed-loop stress test)."""
        torch = self.torch
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reqs = [Request(i, g, np.asarray(s, np.uint32), t0 + (t if realtime else 0.0)) for i, (t, g, s) in
                enumerate(trace)]
        arrivals = collections.deque(reqs)
        pending = {name: collections.deque() for name in self.graphs}
        inflight = []  # (done_event, reqs, bytes, stream)
        free_streams = list(self.streams)
        used = 0
        batch_id = 0
        self.peak_bytes = 0
        while arrivals or inflight or any(pending.values()):
            now = time.perf_counter()
            while arrivals and arrivals[0].arrival <= now:
                r = arrivals.popleft()
                pending[r.graph].append(r)
            still = []
            for ev, rs, nbytes, st in inflight:
                if ev.query():
                    done_at = t0 + ref.elapsed_time(ev) / 1000.0
                    for r in rs:
                        r.done_at = done_at
                    used -= nbytes
                    free_streams.append(st)
                else:
                    still.append((ev, rs, nbytes, st))
            inflight = still
            launched = False
            while free_streams:
                plan = plan_batch(pending, self.budget - used, self.footprint, self.max_k)
                if plan is None:
                    break
                name, take = plan
                for r in take:
                    pending[name].popleft()
                k = sum(r.k for r in take)
                nbytes = self.footprint(name, k)
                st = free_streams.pop()
                ev = self._launch(name, take, st, batch_id)
                batch_id += 1
                used += nbytes
                self.peak_bytes = max(self.peak_bytes, used)
                inflight.append((ev, take, nbytes, st))
                launched = True
            if not launched and not arrivals and not any(pending.values()) and inflight:
                inflight[0][0].synchronize()
            elif not launched:
                time.sleep(20e-6)
        torch.cuda.synchronize()
        self.batches = batch_id
        return reqs


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
