"""Autotuner for the layout and launch settings of a resident graph, with its
choices kept per graph class and size.

The slice width sigma and the slots per lane (tau = 64 * slots) fix the BVSS
layout, so each (sigma, slots) pair is built once; the group depth, the update
scheme (eager, Algorithm 2; lazy, Algorithm 3; adaptive, per level) and the
adaptive threshold are launch settings switched with ``Graph.configure`` on the
same build.  Every candidate runs the given sources
(single-source calls for k = 1, one k-source call otherwise) a few times on one
stream, timed with HIP events, and the fastest median wins.  Each candidate's
levels are compared with the first candidate's, so a tuning run is also a
consistency check across layouts and schemes.

Choices are stored in ``tuned.json`` next to this file under a key made of the
graph class (skewed or mesh-like, from the degree distribution), the size
(log2 of the vertex count) and the source count; ``lookup`` returns the options
for a graph, which the benchmark and the serving loop pass to ``Graph``.

Run: ``python -m paper_2512_21967_amd.autotune --workload rmat22`` (on the GPU).
"""
from __future__ import annotations

import argparse
import dataclasses
import itertools
import json
import math
import os
import sys

import numpy as np

SIGMAS = (8, 16, 32)
SLOTS = (1, 2, 4, 8)
GROUPS = (1, 2, 4)
UPDATES = ("eager", "lazy", "adaptive")
TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


@dataclasses.dataclass
class Trial:
    sigma: int
    slots: int
    group: int
    update: str
    ms: float                      # median over repeats of one round (all sources)
    eager_max: int = 0             # adaptive threshold (0 = the library's default)
    max_grid: int = 0              # cap on the single-source grid (0 = every co-resident workgroup)

    def options(self) -> dict:
        o = {"sigma": self.sigma, "slots": self.slots, "group": self.group, "update": self.update,
             "eager_max": self.eager_max}
        if self.max_grid:
            o["max_grid"] = self.max_grid
        return o


def graph_key(csr, k: int = 1) -> str:
    """'skewed' when the largest degree exceeds 10 times the mean (power-law-like
    graphs), else 'mesh'; then log2 of the vertex count and the source count."""
    deg = np.diff(np.asarray(csr.row_ptr, dtype=np.int64))
    mean = max(float(deg.mean()), 1e-9)
    cls = "skewed" if float(deg.max()) > 10.0 * mean else "mesh"
    return f"{cls}-s{int(round(math.log2(max(int(csr.n), 1))))}-k{'1' if k == 1 else 'multi'}"


def load(path: str = TUNED_PATH) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(csr, k: int = 1, path: str = TUNED_PATH):
    """(key, options) stored for this graph's class and size, or (key, None)."""
    key = graph_key(csr, k)
    rec = load(path).get(key)
    return key, (dict(rec["options"]) if rec else None)


def save(key: str, best: Trial, trials, workload: str, path: str = TUNED_PATH):
    db = load(path)
    db[key] = {"options": best.options(), "ms": round(best.ms, 4), "workload": workload,
               "candidates": [dict(t.options(), ms=round(t.ms, 4)) for t in sorted(trials, key=lambda t: t.ms)]}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(sigmas=SIGMAS, slots=SLOTS, groups=GROUPS, updates=UPDATES, eager_maxes=(0,),
               max_slots_in_flight=16):
    """(sigma, slots, group, update, eager_max) tuples worth timing.  group * slots is
    capped: larger products hold more slice registers than a 1024-thread workgroup
    has without spilling.  Thresholds apply to the adaptive scheme only."""
    out = []
    for sg, sl, gr, up in itertools.product(sigmas, slots, groups, updates):
        if sl * gr > max_slots_in_flight:
            continue
        for em in (eager_maxes if up == "adaptive" else (0,)):
            out.append((sg, sl, gr, up, em))
    return out


def _round(g, sources, k, stream):
    if k == 1:
        return [g.bfs(int(s), stream=stream) for s in sources]
    return [g.bfs_multi(np.asarray(sources, np.uint32), stream=stream)]


def autotune(csr, sources, *, k=1, cands=None, repeats=3, reorder="auto", window=0, device=0, log=None,
             max_grids=(0,)):
    """Times every candidate on `sources` and returns (best Trial, [Trial...]).

    k = 1 times one single-source BFS per source; k > 1 times one k-source call on
    the first k sources.  The builds use the same ordering options, so the
    candidates differ only in layout and launch settings.  max_grids: caps on the
    single-source grid to try with every candidate (a build option; 0 = none)."""
    import torch
    import paper_2512_21967_amd as blest

    cands = candidates() if cands is None else [tuple(c) + (0,) * (5 - len(c)) for c in cands]
    if k > 1:  # the k-source kernel has one update scheme and no group setting
        cands = sorted({(c[0], c[1], 2, "lazy", 0) for c in cands})
    src = [int(s) for s in (sources if k == 1 else list(sources)[:k])]
    stream = torch.cuda.current_stream()
    trials, ref = [], None
    by_layout = {}
    for c in cands:
        for mg in (max_grids if k == 1 else (0,)):
            by_layout.setdefault((c[0], c[1], mg), []).append(c)
    for (sg, sl, mg), group in by_layout.items():
        g = blest.Graph(csr, sigma=sg, slots=sl, window=window - window % sg, reorder=reorder, device=device,
                        max_grid=mg)
        for _, _, gr, up, em in group:
            g.configure(update=up, group=gr, eager_max=em)
            outs = _round(g, src, k, stream)          # warm-up (and workspace allocation)
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
                _round(g, src, k, stream)
                b.record(stream)
                b.synchronize()
                times.append(a.elapsed_time(b))
            t = Trial(sg, sl, gr, up, float(np.median(times)), em, mg)
            trials.append(t)
            if log:
                log(f"[autotune] sigma={sg} slots={sl} group={gr} {up} eager_max={em} max_grid={mg}: {t.ms:.3f} ms")
        g.close()
    best = min(trials, key=lambda t: t.ms)
    return best, trials


# candidate sets of the benchmark workloads (sigma = 8 is the paper's width; the
# orderings take seconds per build at these sizes, so the layouts are few)
WORKLOADS = {
    "rmat22": dict(cands=candidates((8,), (2, 4), (1, 2), ("lazy", "adaptive"), (0, 4096)),
                   k=1, nsrc=16, max_grids=(0, 192, 128)),
    # wider slices for the same class: half the slice sets, 2-byte masks (unpacked)
    "rmat22-wide": dict(cands=candidates((16, 32), (2, 4), (1,), ("lazy", "adaptive"), (0, 4096)),
                        k=1, nsrc=16),
    "grid4096": dict(cands=candidates((8,), (1, 2), (1, 2), ("eager",), (0,)), k=1, nsrc=4, max_grids=(0, 64, 32)),
    "rmat16": dict(cands=candidates((8, 16), (1, 2, 4), (1, 2), UPDATES, (0, 256)), k=1, nsrc=16,
                   max_grids=(0, 128, 64)),
    "rmat20x64": dict(cands=candidates((8, 16, 32), (1, 2, 4), (2,), ("lazy",), (0,)), k=64, nsrc=64),
}


def main():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=sorted(WORKLOADS))
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--out", default=TUNED_PATH, help="store to update (default: the package's tuned.json)")
    args = ap.parse_args()
    w = WORKLOADS[args.workload]
    if args.workload in ("rmat22", "rmat22-wide"):
        gr, reorder = inputs.rmat_workload(22, 16, seed=1, permute_seed=2), "compression"
        src = inputs.sources(gr, seed=3, k=64)[:w["nsrc"]]
    elif args.workload == "grid4096":
        gr, reorder = inputs.grid_workload(4096, 0.9, seed=3, permute_seed=4), "bandwidth"
        src = inputs.sources(gr, seed=5, k=16)[:w["nsrc"]]
    elif args.workload == "rmat16":
        gr, reorder = inputs.rmat_workload(16, 16, seed=1), "none"
        src = inputs.sources(gr, seed=3, k=64)[:w["nsrc"]]
    else:
        gr, reorder = inputs.rmat_workload(20, 16, seed=1), "none"
        src = inputs.sources(gr, seed=7, k=64, distinct=True)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    best, trials = autotune(gr, src, k=w["k"], cands=w["cands"], repeats=args.repeats, reorder=reorder, log=log,
                            max_grids=w.get("max_grids", (0,)))
    key = graph_key(gr, w["k"])
    save(key, best, trials, args.workload, path=args.out)
    print(json.dumps({"key": key, "best": best.options(), "ms": best.ms}), flush=True)


if __name__ == "__main__":
    main()
