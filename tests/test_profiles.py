"""The committed hardware-counter summary belongs to the current step kernel:
its recorded source digest equals the digest of the kernel sources in the
tree (comments and blank space aside), so the benchmark's roofline reports
measured traffic instead of null, and every profile summary names the
command that produced it."""
from __future__ import annotations

from pathlib import Path

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_counter_summary_matches_kernel_sources():
    kv = {}
    for line in (ROOT / bench.TRAFFIC_SUMMARY).read_text().splitlines():
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    assert kv["source_sha256"] == bench.source_digest()
    assert int(kv["traffic_bytes_per_launch"]) >= int(kv["algorithmic_bytes_per_launch"])


def test_every_profile_summary_names_its_command():
    files = sorted((ROOT / "profiles").glob("*.txt"))
    assert len(files) >= 4
    for f in files:
        text = f.read_text()
        assert "rocprofv3 " in text and "python bench.py" in text, f.name
        assert len(text) < 16 * 1024, f.name
