"""bench.py's command line on the host: a request for more than one GPU is
refused before anything runs (this build measures one GPU), and the pinning
flags accept only their documented values.  Nothing here touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "Nothing was run" in r.stderr
    assert r.stdout == ""


def test_pinning_flags_take_zero_or_one():
    for flag in ("--raw-handoff", "--mfma-modup"):
        r = run_bench(flag, "2", "--gpus", "2")
        assert r.returncode == 2
        assert "invalid choice" in r.stderr, flag
