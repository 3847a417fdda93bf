"""The stored digests of the oracle's output (tests/golden/digests.json) agree
with the oracle and the generator as they stand, on the cases cheap enough to
recompute on the host: the tiny workload and the smallest batch instances."""
import hashlib
import json
import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _cases():
    with open(os.path.join(HERE, "golden", "digests.json")) as fh:
        return json.load(fh)["cases"]


def test_tiny_digest_recomputes():
    c = _cases()["tiny"]
    w = synth.workload("tiny")
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    assert _sha(s) == c["input_sha256"]
    assert _sha(oracle.to_int32(oracle.correlate(s)).astype("<i4")) == c["vis_sha256"]


def test_small_batch_instances_recompute():
    c = _cases()["batch"]
    inst = synth.batch_instances()
    assert [(x["N"], x["F"], x["T"]) for x in c["instances"]] == inst
    small = [k for k, (N, F, T) in enumerate(inst) if N <= 128][:3]
    assert small
    for k in small:
        s = synth.batch_frame(k, inst[k])
        assert _sha(s) == c["instances"][k]["input_sha256"], k
        v = oracle.to_int32(oracle.correlate(s)).astype("<i4")
        assert _sha(v) == c["instances"][k]["vis_sha256"], k


def test_every_case_present():
    c = _cases()
    assert set(c) >= {"tiny", "pathfinder", "full_array", "precision_subset", "batch", "stream"}
    assert len(c["batch"]["instances"]) == 48
    assert len(c["stream"]["frames"]) >= 10
