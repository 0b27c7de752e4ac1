"""Autotuner for the launch shape of a resident graph.

The slice width sigma and the slots per lane (tau = 64 * slots) fix the BVSS
layout, so each (sigma, slots) pair is built once; the group depth and the update
scheme (eager, Algorithm 2; lazy, Algorithm 3) are launch settings switched with
``Graph.configure`` on the same build.  Every candidate runs the given sources
(single-source calls for k = 1, one k-source call otherwise) a few times on one
stream, timed with HIP events, and the fastest median wins.  Each candidate's
levels are compared with the first candidate's, so a tuning run is also a
consistency check across layouts.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np

SIGMAS = (8, 16, 32)
SLOTS = (1, 2, 4, 8)
GROUPS = (1, 2, 4)
UPDATES = ("eager", "lazy")


@dataclasses.dataclass
class Trial:
    sigma: int
    slots: int
    group: int
    update: str
    ms: float                      # median over repeats of one round (all sources)

    def options(self) -> dict:
        return {"sigma": self.sigma, "slots": self.slots, "group": self.group, "update": self.update}


def candidates(sigmas=SIGMAS, slots=SLOTS, groups=GROUPS, updates=UPDATES, max_slots_in_flight=16):
    """(sigma, slots, group, update) tuples worth timing.  group * slots is capped:
    larger products hold more slice registers than a 1024-thread workgroup has
    without spilling."""
    out = []
    for sg, sl, gr, up in itertools.product(sigmas, slots, groups, updates):
        if sl * gr <= max_slots_in_flight:
            out.append((sg, sl, gr, up))
    return out


def _round(g, sources, k, stream, torch):
    if k == 1:
        outs = [g.bfs(int(s), stream=stream) for s in sources]
        return outs
    return [g.bfs_multi(np.asarray(sources, np.uint32), stream=stream)]


def autotune(csr, sources, *, k=1, cands=None, repeats=3, reorder="auto", window=1 << 16, device=0, log=None):
    """Times every candidate on `sources` and returns (best Trial, [Trial...]).

    k = 1 times one single-source BFS per source; k > 1 times one k-source call on
    the first k sources.  The builds use the same ordering options, so the
    candidates differ only in layout and launch settings."""
    import torch
    import paper_2512_21967_amd as blest

    cands = candidates() if cands is None else list(cands)
    if k > 1:  # the k-source kernel has one update scheme and no group setting
        cands = sorted({(c[0], c[1], 2, "lazy") for c in cands})
    src = [int(s) for s in (sources if k == 1 else list(sources)[:k])]
    stream = torch.cuda.current_stream()
    trials, ref = [], None
    by_layout = {}
    for c in cands:
        by_layout.setdefault((c[0], c[1]), []).append(c)
    for (sg, sl), group in by_layout.items():
        g = blest.Graph(csr, sigma=sg, slots=sl, window=window - window % sg, reorder=reorder, device=device)
        for _, _, gr, up in group:
            g.configure(update=up, group=gr)
            outs = _round(g, src, k, stream, torch)          # warm-up (and workspace allocation)
            torch.cuda.synchronize()
            got = [o.cpu().numpy() for o in outs]
            if ref is None:
                ref = got
            elif not all(np.array_equal(a, b) for a, b in zip(ref, got)):
                raise RuntimeError(f"levels differ between layouts at sigma={sg} slots={sl} group={gr} {up}")
            times = []
            for _ in range(repeats):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                _round(g, src, k, stream, torch)
                b.record(stream)
                b.synchronize()
                times.append(a.elapsed_time(b))
            t = Trial(sg, sl, gr, up, float(np.median(times)))
            trials.append(t)
            if log:
                log(f"[autotune] sigma={sg} slots={sl} group={gr} {up}: {t.ms:.3f} ms")
        g.close()
    best = min(trials, key=lambda t: t.ms)
    return best, trials
