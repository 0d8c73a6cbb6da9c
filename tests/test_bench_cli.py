"""bench.py's command-line contract on the CPU: more than one GPU is refused with a JSON message
and a non-zero status, and without a visible GPU the run stops with a JSON message instead of
falling back to anything else."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=timeout, cwd=ROOT)


def test_several_gpus_are_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_no_gpu_stops_the_run():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = _run("--no-cpu-baseline", "--leg", "uneven", "--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert json.loads(r.stdout.strip().splitlines()[-1]) == {"error": "no GPU visible"}


def test_flops_per_pair_of_the_network():
    # 6 -> [width] x depth -> 7, two flops per multiply-add
    sys.path.insert(0, ROOT)
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_cli_probe", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    assert b.mlp_flops_per_pair(64, 4) == 2 * (6 * 64 + 3 * 64 * 64 + 64 * 7)
    assert b.mlp_flops_per_pair(256, 4) == 2 * (6 * 256 + 3 * 256 * 256 + 256 * 7)
    assert b.mlp_flops_per_pair() == b.mlp_flops_per_pair(b.MLP_WIDTH, b.MLP_DEPTH)
