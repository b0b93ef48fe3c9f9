"""bench.py's command-line contract on a machine without a GPU: one GPU only
(other counts exit with a message), and a clear exit when no HIP device is
present, for every workload."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("workload", ["c3", "c4", "c5", "lossless"])
def test_no_device_exits_cleanly(workload):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    r = run("--workload", workload, "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "needs a HIP device" in r.stderr
