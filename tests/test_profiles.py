"""The benchmark reports measured HBM traffic only for the kernel the
counters were taken on: when the recorded source digest of the committed
counter summary equals the digest of the kernel sources in the tree (comments
and blank space aside) the traffic is at least the algorithmic bytes;
otherwise the benchmark reports null with the reason.  Every profile summary
names the command that produced it."""
from __future__ import annotations

import json
from pathlib import Path

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_traffic_is_reported_only_for_the_profiled_kernel():
    for rel, key, reader in ((bench.TRAFFIC_SUMMARY, "traffic_bytes_per_launch", bench.measured_traffic),
                             (bench.ISSUE_SUMMARY, "valu_issue_frac", bench.measured_issue)):
        kv = bench.read_summary(rel)
        if kv is None:
            assert reader({})[0] is None
            continue
        value, why = reader(json.loads(kv["tuning"]))
        if kv["source_sha256"] == bench.source_digest():
            assert value == type(value)(kv[key])
            if key == "traffic_bytes_per_launch":
                assert value >= int(kv["algorithmic_bytes_per_launch"])
        else:
            assert value is None and "changed" in why


def test_every_profile_summary_names_its_command():
    files = sorted((ROOT / "profiles").glob("*.txt"))
    assert len(files) >= 4
    for f in files:
        text = f.read_text()
        assert "rocprofv3 " in text and "python bench.py" in text, f.name
        assert len(text) < 16 * 1024, f.name
