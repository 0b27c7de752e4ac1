"""Summaries of rocprofv3 output for the committed profile records.

  python -m paper_2512_21967_amd.profsum stats DIR --cmd "<command>" > profiles/<kernel>_<workload>.txt
      Kernel table (calls, total, average, min, max) from the *_kernel_stats.csv
      that `rocprofv3 --kernel-trace --stats --output-format csv -d DIR` wrote.

  python -m paper_2512_21967_amd.profsum traffic FETCH_DIR WRITE_DIR --key rmat22/lazy \
        --kernel bfs_persistent --copy-bytes 268435456 --cmd-fetch "..." --cmd-write "..."
      HBM traffic per launch of the named kernel from one `--pmc FETCH_SIZE` run and
      one `--pmc WRITE_SIZE` run, each scaled by what the same counter read for the
      plain device copy of --copy-bytes (read once, written once) that the profiled
      command ran after its timed region.  Merges the record into
      profiles/traffic.json under --key, stamped with the hash of the csrc files the
      kernel is built from (--sources; by default the single-source kernel's), so
      that a later change to any of them voids it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


CSRC = os.path.join(ROOT, "paper_2512_21967_amd", "csrc")
# Sources that build the single-source kernel and everything it reads or is
# launched with (host-side layout, options, launch shape); the other kernels live
# in translation units of their own and cannot change its code or traffic.
SINGLE_SOURCE_FILES = ("bfs_kernel.hpp", "capi.cpp", "device_common.hpp", "host.cpp", "internal.hpp", "kernels.hip",
                       "kernels.hpp", "kernels_adaptive.hip", "kernels_eager.hip", "kernels_lazy.hip")


def kernel_source_hash(files=None):
    """Hash of the named csrc files (all of them when files is None)."""
    if files is None:
        paths = [f for f in sorted(glob.glob(os.path.join(CSRC, "*"))) if f.endswith((".hip", ".hpp", ".cpp"))]
    else:
        paths = [os.path.join(CSRC, f) for f in sorted(files)]
    h = hashlib.sha256()
    for f in paths:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits


def _short(name, width=110):
    name = " ".join(name.split())
    return name if len(name) <= width else name[:width - 3] + "..."


def stats(args):
    rows = []
    for f in _find(args.dir, "kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"# rocprofv3 kernel statistics\n# command: {args.cmd}\n")
    print(f"{'calls':>7} {'total ms':>10} {'avg us':>10} {'min us':>10} {'max us':>10} {'%':>6}  kernel")
    for r in rows:
        print(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}  "
              f"{_short(r['Name'])}")


def _counter(d, counter):
    """[(kernel_name, value)] per dispatch, in dispatch order."""
    per = {}
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                key = (f, int(r["Dispatch_Id"]))
                name, val = per.get(key, (r["Kernel_Name"], 0.0))
                per[key] = (name, val + float(r["Counter_Value"]))
    return [per[k] for k in sorted(per)]


def _scaled(d, counter, kernel, copy_kib):
    rows = _counter(d, counter)
    copy = [v for n, v in rows if "copy" in n.lower() or "elementwise" in n.lower()]
    calib = [v for v in copy if v > 0.5 * copy_kib]
    if not calib:
        raise SystemExit(f"{counter}: no copy dispatch of about {copy_kib:.0f} KiB found for calibration")
    factor = copy_kib / calib[-1]
    mine = [v for n, v in rows if kernel in n]
    if not mine:
        raise SystemExit(f"{counter}: no dispatch of {kernel}")
    return sum(mine) / len(mine) * 1024.0 * factor, factor, len(mine)


def traffic(args):
    copy_kib = args.copy_bytes / 1024.0
    fetch, ff, nf = _scaled(args.fetch_dir, "FETCH_SIZE", args.kernel, copy_kib)
    write, fw, nw = _scaled(args.write_dir, "WRITE_SIZE", args.kernel, copy_kib)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    db = {}
    if os.path.exists(path):
        with open(path) as f:
            db = json.load(f)
    db[args.key] = {"bytes_per_launch": round(fetch + write), "fetch_bytes_per_launch": round(fetch),
                    "write_bytes_per_launch": round(write), "fetch_scale": round(ff, 4), "write_scale": round(fw, 4),
                    "dispatches": [nf, nw], "kernel": args.kernel, "kernel_sources": sorted(args.sources),
                    "kernel_source_hash": kernel_source_hash(args.sources),
                    "commands": [args.cmd_fetch, args.cmd_write]}
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(db[args.key], indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--key", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=float, default=float(256 << 20))
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--sources", nargs="+", default=list(SINGLE_SOURCE_FILES),
                   help="csrc files whose hash stamps the record (default: the single-source kernel's)")
    args = ap.parse_args(argv)
    stats(args) if args.what == "stats" else traffic(args)


if __name__ == "__main__":
    main(sys.argv[1:])
