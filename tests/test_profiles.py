"""The benchmark reports measured HBM traffic only for the kernel the
counters were taken on: when the recorded source digest of the committed
counter summary equals the digest of the kernel sources in the tree (comments
and blank space aside) the traffic is at least the algorithmic bytes;
otherwise the benchmark reports null with the reason.  Every profile summary
names the command that produced it."""
from __future__ import annotations

from pathlib import Path

import bench

ROOT = Path(__file__).resolve().parents[1]


def _summary():
    kv = {}
    for line in (ROOT / bench.TRAFFIC_SUMMARY).read_text().splitlines():
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_is_reported_only_for_the_profiled_kernel():
    kv = _summary()
    traffic, why = bench.measured_traffic(__import__("json").loads(kv["tuning"]))
    if kv["source_sha256"] == bench.source_digest():
        assert traffic == int(kv["traffic_bytes_per_launch"])
        assert traffic >= int(kv["algorithmic_bytes_per_launch"])
    else:
        assert traffic is None and "changed" in why


def test_every_profile_summary_names_its_command():
    files = sorted((ROOT / "profiles").glob("*.txt"))
    assert len(files) >= 4
    for f in files:
        text = f.read_text()
        assert "rocprofv3 " in text and "python bench.py" in text, f.name
        assert len(text) < 16 * 1024, f.name
