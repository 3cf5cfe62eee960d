"""Host logic of bench.py (no GPU): the one-GPU rule, the roofline arithmetic, the counter
lookup guarded by the source hash."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "only --gpus 1" in line["error"]


def test_roofline_takes_the_dominant_pass_family():
    sb = 1 << 28                                    # 256 MiB state
    stats = {"tile_low": (500, 500 * 0.088), "tile_high": (500, 500 * 0.0968),
             "reduce_flip": (4, 10.0), "init": (1, 0.04)}
    r = bench.roofline_from_stats(stats, sb, None)
    assert r["kernel"] == "tile_high" and r["launches"] == 500
    assert r["avg_us"] == pytest.approx(96.8)
    # two state-sized transfers per launch over the mean launch time
    assert r["achieved"] == pytest.approx(2 * sb / 96.8e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["state_in_memory"].startswith("the size of the Infinity Cache")
    assert bench.roofline_from_stats({"init": (1, 1.0)}, sb, None) is None


def test_state_residency_labels():
    assert bench.cache_residency(128 << 20) == "resident in the Infinity Cache"
    assert bench.cache_residency(32 << 30) == "streams HBM"


def test_counter_lookup_needs_matching_sources(tmp_path, monkeypatch):
    here = bench.kernel_source_hash()
    assert len(here) == 16
    d = {"source_hash": "0" * 16, "kernels": {"c128:2x2x2:tile_high": {"hbm_bytes_per_launch": 1.0}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: here)
    assert bench.load_traffic("c128:2x2x2:tile_high") is None       # other sources
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("c128:2x2x2:tile_high") == 1.0
    assert bench.load_traffic("c64:2x2x2:tile_high") is None
