"""Command-line contract of bench.py that needs no GPU: more than one GPU is
refused with a message before anything touches a device, and the help lists
every workload."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_help_lists_the_workloads():
    r = run_bench("--help")
    assert r.returncode == 0
    for name in ("c3", "c4", "section5"):
        assert name in r.stdout
