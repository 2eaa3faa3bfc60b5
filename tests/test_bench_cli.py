"""The bench's argument contract, checked without a GPU: more than one GPU is refused with a
message (this build measures one GPU), and so is a timed loop with no solve in flight."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_inflight_must_be_positive():
    r = _run("--inflight", "0")
    assert r.returncode != 0
    assert "--inflight" in r.stderr and r.stdout == ""
