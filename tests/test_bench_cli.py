"""The benchmark's command-line contract that needs no GPU: more than one
GPU is refused with a JSON message and a non-zero status, and the help
text lists the workloads."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("single", "batched", "steploop", "copy"):
        assert w in r.stdout
