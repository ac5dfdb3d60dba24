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
