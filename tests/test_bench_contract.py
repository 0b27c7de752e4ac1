"""Host-side checks of bench.py's command-line contract (no GPU): more than one GPU
is refused with a message, every workload name parses, and the roofline record
reports traffic only for profiles taken on the current kernel sources."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_fields():
    roof = bench.roofline(1.0e9, 0.5e-3, "no-such-profile")
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["achieved"] - 2000.0) < 1e-6 and abs(roof["frac"] - 0.25) < 1e-9
    assert roof["traffic"] is None


def test_committed_traffic_records_match_their_sources():
    """Each committed record names the sources it was taken on; bench.py reports its
    bytes only while their hash still matches."""
    from paper_2512_21967_amd import profsum
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        db = json.load(f)
    for key, rec in db.items():
        assert rec["bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"] or \
            abs(rec["bytes_per_launch"] - rec["fetch_bytes_per_launch"] - rec["write_bytes_per_launch"]) <= 1
        want = rec["bytes_per_launch"] if rec["kernel_source_hash"] == profsum.kernel_source_hash(
            rec.get("kernel_sources")) else None
        assert bench.traffic_from_profiles(key) == want
