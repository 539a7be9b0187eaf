"""Command-line contract of bench.py that holds without a GPU: it measures
one GPU only, and says so for any other count before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = run_bench("--gpus", n)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_several_ranks_are_refused():
    env = dict(os.environ, WORLD_SIZE="2", RANK="0", LOCAL_RANK="0")
    r = run_bench(env=env)
    assert r.returncode == 2
    assert "WORLD_SIZE" in r.stderr and r.stdout == ""
