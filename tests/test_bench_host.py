"""Host checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message, and --help lists the legs."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
    assert "--gpus 1" in r.stderr


def test_help_lists_every_leg():
    r = run("--help")
    assert r.returncode == 0
    for leg in ("parity", "sweep", "split", "batched", "batched_plan", "tuner", "memory"):
        assert leg in r.stdout
