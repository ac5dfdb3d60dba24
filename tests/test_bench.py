"""Host-side parts of bench.py (no GPU): the refusal of several GPUs, the
build's compulsory-bytes figure and the reading of the committed counter
summaries."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1606_07550_amd import profiling  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_build_line_counts_each_compulsory_byte_once():
    n, m_raw, m = 10, 40, 30
    b = bench.build_line(2.0, n, m_raw, m)
    # pairs read once; symmetric rows, DAG out- and in-lists written once;
    # three offset arrays and three degree arrays
    assert b["compulsory_bytes"] == 8 * m_raw + 4 * 2 * m + 4 * m + 4 * m + 3 * 8 * (n + 1) + 3 * 4 * n
    assert b["GBps"] == pytest.approx(b["compulsory_bytes"] / 2e-3 / 1e9)
    assert b["frac"] == pytest.approx(b["GBps"] / bench.HBM_PEAK_GBPS)
    assert bench.build_line(0.0, n, m_raw, m)["GBps"] == 0.0


@pytest.mark.parametrize("name", ["counters_rmat24.md", "counters_batch4096.md"])
def test_counter_summaries_parse(name):
    rec = profiling.read_summary(os.path.join(ROOT, "profiles", name))
    for key in ("kernel", "variant", "workload", "traffic_bytes_per_launch", "dram_bytes_per_launch",
                "l2_hit_rate", "count_kernels_sha256"):
        assert key in rec, key
    assert 0.0 <= float(rec["l2_hit_rate"]) <= 1.0
    assert float(rec["dram_bytes_per_launch"]) > 0


def test_launch_groups_follow_equal_adjacent_variants():
    assert bench.launch_groups([21, 23, 24, 20, 20, 9]) == [(0, 0), (1, 1), (2, 2), (3, 4), (5, 5)]
    assert bench.launch_groups([1, 1, 1, 1, 1, 1]) == [(0, 5)]
    assert bench.launch_groups([0, 1, 0, 1, 0, 1]) == [(b, b) for b in range(6)]
    assert bench.launch_groups([10, 10, 11, 12, 12, 8]) == [(0, 1), (2, 2), (3, 4), (5, 5)]


def test_counters_are_used_only_for_their_launch(monkeypatch):
    rec = {"count_kernels_sha256": profiling.count_source_sha256(), "variant": "20", "bin": "3-4",
           "traffic_bytes_per_launch": "100", "dram_bytes_per_launch": "120", "l2_hit_rate": "0.05"}
    monkeypatch.setattr(profiling, "read_summary", lambda path: dict(rec))
    got = bench.measured_counters("rmat24", 20, "3-4")
    assert got["traffic_bytes_per_launch"] == 100.0 and got["l2_hit_rate"] == 0.05
    assert bench.measured_counters("rmat24", 20, "3") is None  # another launch
    assert bench.measured_counters("rmat24", 21, "3-4") is None  # another variant
    rec["count_kernels_sha256"] = "0" * 64  # taken on another kernel source
    assert bench.measured_counters("rmat24", 20, "3-4") is None


def test_summary_names_the_dispatches_it_averages():
    assert "bins 3-4" in profiling._selection("3-4", 1, 0)
    assert "bin 3's launches" in profiling._selection(3, 2, 0)
    assert profiling._selection(None, 1, 0) == ""
