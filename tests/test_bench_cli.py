"""The benchmark's command line refuses what it cannot measure (CPU, no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    return r.returncode, r.stdout.strip().splitlines()


def test_more_than_one_gpu_is_refused_with_a_message():
    rc, out = _run("--gpus", "2")
    assert rc == 2
    msg = json.loads(out[-1])
    assert "--gpus must be 1" in msg["error"]


def test_no_visible_gpu_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible here")
    rc, out = _run("--steps", "1", "--warmup", "0")
    assert rc == 2
    assert json.loads(out[-1]) == {"error": "no GPU visible"}
