"""GPU: bench.py's one JSON line, as the benchmark contract defines it,
from short runs of the headline workload and of one VALU configuration."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
QUIET = ["--no-server", "--no-cpu", "--no-vendor", "--no-peaks", "--no-graph", "--no-configs"]


def bench_line(*args):
    print("case: bench.py " + " ".join(args), flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.strip().splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0])


def test_headline_line_fields():
    d = bench_line("--steps", "3", "--warmup", "2", *QUIET)
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 2
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["scaling"] == "weak" and d["vs_baseline"] is None and d["data"] == "synthetic"
    assert d["dtype"] == "bf16x3" and d["config"]["workload"] == "ring_longk"
    rf = d["roofline"]
    assert rf["bound"] == "mfma" and rf["unit"] == "TFLOP/s" and rf["peak"] == 2500.0
    assert 0 < rf["achieved"] < rf["peak"] and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    # the kernel's time sits inside the step's
    assert rf["kernel_ms"] <= d["ms_per_step"] * 1.02
    assert d["error"]["ok"] and d["error"]["log2"] < -20
    grid = d["grid_baseline"]
    assert grid["ms_per_step"] > 0 and grid["default_ms"] > 0 and grid["trials"] > 1
    assert abs(d["paco_vs_grid"] - grid["ms_per_step"] / grid["paco_ms_compared"]) < 1e-3


def test_valu_workload_line_fields():
    d = bench_line("--workload", "minplus_c0", "--steps", "20", "--warmup", "5", *QUIET)
    assert d["dtype"] == "u32" and d["config"]["workload"] == "minplus_c0"
    rf = d["roofline"]
    assert rf["bound"] == "alu" and rf["peak"] == 39.3 and rf["achieved"] > 0
    assert d["paco_vs_grid"] > 0 and d["grid_baseline"]["split_k"] >= 1
