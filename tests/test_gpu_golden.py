"""Whole-output parity on the benchmark workloads.

The HIP path's entire int32 output, every baseline of every channel, is
hashed and compared with SHA-256 digests of the oracle's output on the same
seeded inputs (``tests/golden/digests.json``, written by
``tests/golden/make_digests.py``, which calls only the oracle and the
generator).  The definition is that of the X-engine (Sec. I; Sec. IV-C,
"Full Correlation"; Eq. (1)); the integer result is unique, so the HIP path
must match bit for bit in every form and schedule.

Each case first checks the digest of its generated input, so that a
generator drawing other samples is told apart from a wrong correlation.  On
a mismatch the test compares sampled baselines with the oracle to report how
many differ.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1503_06202_amd import BatchPlan, Plan, vis_shape
from paper_1503_06202_amd.stream import Frame, GpuLauncher, RequestLoop, poisson_arrivals

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "digests.json")) as _fh:
    CASES = json.load(_fh)["cases"]


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def vis_sha(v: np.ndarray) -> str:
    assert v.dtype == np.int32
    return sha(v.astype("<i4"))


def check(samples: np.ndarray, got: np.ndarray, want: str, label: str) -> None:
    """Digest of the whole output; on a mismatch, a sampled diff for the report."""
    if vis_sha(got) == want:
        return
    T, F, N = samples.shape
    rng = np.random.default_rng(0)
    n = 400
    f = rng.integers(0, F, n)
    i = rng.integers(0, N, n)
    j = rng.integers(0, N, n)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    ref = oracle.correlate_pairs(samples, f, lo, hi)
    b = lo * N - lo * (lo - 1) // 2 + (hi - lo)
    bad = int((got[f, b].astype(np.int64) != ref).any(axis=1).sum())
    pytest.fail(f"{label}: output digest differs from the oracle's; "
                f"{bad} of {n} sampled baselines differ")


def workload_frame(name, case):
    w = synth.workload(name)
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    assert sha(s) == case["input_sha256"], f"{name}: the generator drew other samples"
    return s


def correlate(s, form):
    T, F, N = s.shape
    d = torch.from_numpy(s).to(DEV)
    with Plan(N, F, T, form=form) as p:
        out = p.correlate(d)
        torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def frames():
    return {}


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("name", ["tiny", "pathfinder", "full_array"])
def test_workload_whole_output(frames, name, form):
    case = CASES[name]
    if name not in frames:
        frames.clear()  # keep one frame in host memory at a time
        frames[name] = workload_frame(name, case)
    s = frames[name]
    print(f"golden {name} N={case['N']} F={case['F']} T={case['T']} form={form}", flush=True)
    check(s, correlate(s, form), case["vis_sha256"], f"{name} {form}")


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_precision_subset_whole_output(frames, form):
    case = CASES["precision_subset"]
    if "precision" not in frames:
        frames.clear()
        w = synth.workload("precision")
        s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind, channels=case["channels"])
        assert sha(s) == case["input_sha256"]
        frames["precision"] = s
    s = frames["precision"]
    print(f"golden precision channels {case['channels']} T={case['T']} form={form}", flush=True)
    check(s, correlate(s, form), case["vis_sha256"], f"precision {form}")


def test_batch_48_instances_whole_output(frames):
    frames.clear()
    case = CASES["batch"]
    inst = synth.batch_instances()
    assert [(x["N"], x["F"], x["T"]) for x in case["instances"]] == inst
    host = [synth.batch_frame(i, x) for i, x in enumerate(inst)]
    for k, h in enumerate(host):
        assert sha(h) == case["instances"][k]["input_sha256"], k
    d = [torch.from_numpy(h).to(DEV) for h in host]
    vis = [torch.full(vis_shape(N, F), -1, dtype=torch.int32, device=DEV) for N, F, T in inst]
    print(f"golden batch of {len(inst)} instances (one persistent launch, graph)", flush=True)
    with BatchPlan(inst) as bp:
        for rep in range(2):  # the second run replays the captured graph
            bp.correlate(d, vis, graph=True)
            torch.cuda.synchronize()
            for k, h in enumerate(host):
                check(h, vis[k].cpu().numpy(), case["instances"][k]["vis_sha256"],
                      f"batch instance {k} {inst[k]} run {rep}")
            for v in vis:
                v.fill_(-1)


def test_stream_frames_alone_and_integrated(frames):
    frames.clear()
    case = CASES["stream"]
    w = synth.workload("stream_frame")
    host = [synth.stream_frame(x["k"]) for x in case["frames"]]
    for h, x in zip(host, case["frames"]):
        assert sha(h) == x["input_sha256"], x["k"]
    d = [torch.from_numpy(h).to(DEV) for h in host]
    print(f"golden stream: {len(d)} frames N={w.N} F={w.F} T={w.T}", flush=True)
    # each frame alone
    with Plan(w.N, w.F, w.T) as p:
        for h, x, t in zip(host, case["frames"], d):
            check(h, p.correlate(t).cpu().numpy(), x["vis_sha256"], f"stream frame {x['k']}")
    # all of them through the request loop: Poisson arrivals, continuous
    # batching into one device accumulator, dumped once the ten have added
    n = len(d)
    arr = poisson_arrivals(n, 2000.0, 11)
    la = GpuLauncher(w.N, w.F, w.T, slots=4, streams=1, graph=True)
    try:
        rep = RequestLoop(la, max_inflight=2, dump_every=n).run(
            [Frame(k, 0, d[k], float(arr[k])) for k in range(n)])
        torch.cuda.synchronize()
        assert rep.frames == n and len(rep.dumps) == 1
        _, count, (_, hostbuf, ev) = rep.dumps[0]
        ev.synchronize()
        assert count == n
        got = hostbuf.numpy()
        assert vis_sha(got) == case["sum_vis_sha256"], "integrated stream differs from the oracle's sum"
        assert not la.acc[0].any().item()  # cleared after the dump
    finally:
        la.close()
