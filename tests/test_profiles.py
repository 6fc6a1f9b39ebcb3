"""Committed HBM-traffic summaries: each names the kernel source it was
measured on; the bench reports its bytes only while that source is
unchanged, so a stale summary must be refreshed, not silently dropped."""
import glob
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md")))


def test_traffic_summaries_exist():
    names = {os.path.basename(p)[:-len("_hbm_traffic.md")] for p in SUMMARIES}
    assert {"ring_longk", "maxplus_c2a", "minplus_8192", "bool_c2b"} <= names


@pytest.mark.parametrize("path", SUMMARIES, ids=os.path.basename)
def test_traffic_summary_matches_current_kernel(path):
    workload = os.path.basename(path)[:-len("_hbm_traffic.md")]
    assert workload in bench.WORKLOADS
    text = open(path).read()
    assert f"workload: {workload}" in text
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    t = bench.measured_traffic(workload)
    assert t is not None, "kernel source changed since the counters were taken"
    assert t > 0
