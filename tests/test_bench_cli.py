"""bench.py's command line on the host: it runs on one GPU only, so more
than one is refused with a message before anything touches a device, and
every workload it offers is listed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_help_lists_every_workload():
    sys.path.insert(0, ROOT)
    import bench
    r = run_bench("--help")
    assert r.returncode == 0
    text = "".join(r.stdout.split())
    for name in bench.WORKLOADS:
        assert name in text
    assert "ring_longk" in bench.WORKLOADS
