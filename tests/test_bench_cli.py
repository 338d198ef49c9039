"""The benchmark's command line on the host (no GPU is touched): the
single-GPU contract and the option set the measurements document."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120,
                          cwd=ROOT, env=env)


@pytest.mark.parametrize("n", ["2", "8"])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = _run("--gpus", n)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_launcher_world_size_is_refused_too():
    env = dict(os.environ, WORLD_SIZE="2")
    r = _run(env=env)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("eloc", "grad", "multi", "sweep", "sample", "vmc"):
        assert w in r.stdout
    for opt in ("--steps", "--warmup", "--batch", "--no-cpu-baseline",
                "--tuning-cache", "--copy-probe-mib"):
        assert opt in r.stdout
