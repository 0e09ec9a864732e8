"""CPU checks of the benchmark's command-line contract: one GPU only, a JSON error
line and a non-zero exit where it cannot run, and the recorded counter traffic
keyed to the step-kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def last_json(out):
    lines = [l for l in out.splitlines() if l.startswith("{")]
    assert lines, out
    return json.loads(lines[-1])


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in last_json(r.stdout)["error"]


def test_no_gpu_is_an_error_not_a_fallback():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "error" in last_json(r.stdout)


def test_recorded_traffic_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench

    assert bench.kernel_hash() in bench.MEASURED_TRAFFIC
