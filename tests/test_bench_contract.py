"""The benchmark's arithmetic on the CPU: the roofline of a launch counts
2 x 9 x sizeof(storage) bytes per species-site-step (every population read
and written once per step) times the species-site-steps one launch advances,
against the MI355X's 8 TB/s; the timing summary reports the median window;
a run asking for more than one GPU is refused with a message."""
from __future__ import annotations

import json
import subprocess
import sys
from pathlib import Path

import pytest

import bench

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.parametrize("storage,b", [("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)])
def test_bytes_per_species_site_step(storage, b):
    r = bench.roofline(1, 1, storage, 1, 1.0, "k")
    assert r["bytes_per_species_site_step"] == 18 * b
    assert r["algorithmic_bytes_per_launch"] == 18 * b


def test_headline_roofline_by_hand():
    # 4096^2 sites, two species, FP32, ten steps per launch, 609.4 us a launch:
    # 72 B x 2 x 16777216 x 10 = 24159191040 B -> 39.644 TB/s, 4.955 of 8 TB/s
    r = bench.roofline(2, 4096 * 4096, "f32", 10, 609.4e-6, "k_stepW")
    assert r["species_site_steps_per_launch"] == 335544320
    assert r["algorithmic_bytes_per_launch"] == 24159191040
    assert r["achieved"] == pytest.approx(39644.2, abs=0.1)
    assert r["frac"] == pytest.approx(4.9555, abs=1e-4)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert r["traffic"] is None
    # measured traffic: GB/s and fraction of the peak over the same launch
    t = bench.roofline(2, 4096 * 4096, "f32", 10, 609.4e-6, "k_stepW", traffic=2514175477, traffic_src="x")
    assert t["hbm_measured_GBs"] == pytest.approx(2514175477 / 609.4e-6 / 1e9, abs=0.1)
    assert t["hbm_measured_frac"] == pytest.approx(2514175477 / 609.4e-6 / 8e12, abs=1e-4)


def test_window_stats_reports_the_median():
    med, st = bench.window_stats([3.0, 1.0, 2.0, 10.0, 2.5], 100)
    assert med == 2.5
    assert st["windows"] == 5 and st["steps_per_window"] == 100
    assert st["min_ms"] == 1000.0 and st["max_ms"] == 10000.0
    assert st["spread_pct"] == pytest.approx((10.0 - 1.0) / 2.5 * 100)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode != 0
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    assert r.returncode == 2 and "one GPU" in json.loads(line)["error"]
