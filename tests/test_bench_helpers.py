"""The measurement arithmetic of bench.py on the host: the DTW roofline (algorithmic band cells of
the lane launches over their time, against 39.3e12 lane-ops/s at three lane-operations per cell),
and the counter summary it attaches (only while the summarised kernels' sources still hash the
same)."""
import importlib.util
import os
import shutil
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench(root=ROOT):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    b.ROOT = root
    return b


def test_dtw_peak_is_the_valu_lane_rate_over_three():
    b = load_bench()
    assert b.VALU_LANE_OPS == pytest.approx(256 * 4 * 16 * 2.4e9)
    assert b.DTW_PEAK_GCUPS == pytest.approx(13107.2, rel=1e-6)


def test_roofline_of_dtw_counts_lane_cells_only():
    b = load_bench(tempfile.mkdtemp())   # no profiles: traffic is None
    meas = {"kernel_ms": {"dtw": [400.0, 2], "lb": [300.0, 2], "dtw_wave": [10.0, 3]},
            "counters": {"dtw_cells": 5_000_000_000_000, "dtw_wave_cells": 1_000_000_000_000},
            "schedule": {"dtw_rows": 1, "lb_tile": 0}, "workload_key": "motifs1e9"}
    r = b.roofline_of(meas)
    cells = 4_000_000_000_000          # the one-wave kernels' cells are not the lane launches'
    assert r["achieved"] == pytest.approx(cells / 0.4 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 13107.2, rel=1e-3)
    assert r["algorithmic_cells_per_launch"] == cells // 2
    assert r["avg_launch_ms"] == pytest.approx(200.0)
    assert r["traffic"] is None and r["bound"] == "alu"


def test_traffic_summary_is_dropped_when_sources_change():
    d = tempfile.mkdtemp()
    os.makedirs(os.path.join(d, "profiles"))
    os.makedirs(os.path.join(d, "src"))
    src = os.path.join(d, "src", "k.hip")
    open(src, "w").write("kernel body\n")
    import hashlib
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    open(os.path.join(d, "profiles", "traffic_k_demo_wl.txt"), "w").write(
        f"# comment = ignored\nkernel = k\nsources = src/k.hip\nsources_sha256 = {sha}\nbytes_per_launch = 1234\n")
    b = load_bench(d)
    assert b.traffic_of("k_demo", "wl") == 1234.0
    assert b.traffic_of("k_other", "wl") is None
    open(src, "w").write("kernel body, changed\n")
    assert b.traffic_of("k_demo", "wl") is None
    shutil.rmtree(d)

