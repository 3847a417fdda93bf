"""Host logic of bench.py: the one-GPU rule of its command line and the shape
of its CPU-baseline object (no GPU needed)."""
import json
import os
import subprocess
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def run_bench(args, env_extra=None):
    env = dict(os.environ, **(env_extra or {}))
    return subprocess.run([sys.executable, BENCH] + args, capture_output=True, text=True, env=env,
                          cwd=ROOT, timeout=300)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None), (["--gpus", "8"], None),
                                      ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(args, env):
    res = run_bench(args, env)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""          # no JSON line for a run that did not happen


def test_no_gpu_is_an_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    res = run_bench(["--forms", "", "--no-cpu-baseline", "--no-ceiling", "--steps", "1"])
    assert res.returncode == 1
    assert "needs a GPU" in res.stderr


def test_cpu_baseline_object():
    sys.path.insert(0, ROOT)
    import bench

    T, F, N = 512, 3, 64
    w = types.SimpleNamespace(T=T, N=N, F=F, baselines=N * (N + 1) // 2, name="test")
    frame = np.random.default_rng(5).integers(0, 256, (T, F, N), dtype=np.uint8)
    out = bench.cpu_baseline(frame, w, budget_s=0.0)
    assert out["kind"] == "oracle" and out["unit"] == "cMAC/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "channels 0..0" in out["sample"]   # a zero budget still runs one whole channel
    one = out["one_core"]
    assert one["cores"] == 1 and one["value"] > 0, one
    json.dumps(out)                           # it goes into the JSON line as is
