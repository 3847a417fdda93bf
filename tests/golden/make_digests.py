"""Write SHA-256 digests of the oracle's full output on the benchmark workloads.

The GPU tests hash the HIP path's whole output on the same seeded inputs and
compare the hashes with these, so that every baseline of every channel of
these workloads is checked bit for bit, at sizes where keeping the oracle's
output itself in the repository would be impractical (the full-array frame's
visibilities are 256 MiB).

The output is the definition of the X-engine (Sec. I; Sec. IV-C, "Full
Correlation"; Eq. (1)): int32 [F][N(N+1)/2][2] as the oracle computes it,
hashed as its little-endian bytes in C order.  Each case also records the
SHA-256 of its input bytes, so that a generator that drew different samples
is told apart from a correlation that went wrong.

This script calls only ``oracle/`` and ``synth/``.  Run it from the
repository root (about 15 minutes on 8 host cores):

    python tests/golden/make_digests.py            # every case
    python tests/golden/make_digests.py --only full_array
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "digests.json")

STREAM_FRAMES = 10      # frames 0..9 of the streaming workload, and their sum
PRECISION_CHANNELS = (0, 1)


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def vis_digest(v64: np.ndarray) -> str:
    """Digest of an oracle result as the int32 output type (little-endian)."""
    v = oracle.to_int32(v64)
    return sha(v.astype("<i4"))


def case_workload(name: str) -> dict:
    w = synth.workload(name)
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    return {"N": w.N, "F": w.F, "T": w.T, "recipe": w.kind, "seed": w.seed,
            "input_sha256": sha(s), "vis_sha256": vis_digest(oracle.correlate(s))}


def case_precision() -> dict:
    w = synth.workload("precision")
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind, channels=list(PRECISION_CHANNELS))
    return {"N": w.N, "F": w.F, "T": w.T, "recipe": w.kind, "seed": w.seed,
            "channels": list(PRECISION_CHANNELS), "input_sha256": sha(s),
            "vis_sha256": vis_digest(oracle.correlate(s))}


def case_batch() -> dict:
    inst = synth.batch_instances()
    out = []
    for i, x in enumerate(inst):
        s = synth.batch_frame(i, x)
        out.append({"N": x[0], "F": x[1], "T": x[2], "input_sha256": sha(s),
                    "vis_sha256": vis_digest(oracle.correlate(s))})
    return {"count": len(inst), "seed": 5, "recipe": "gauss", "instances": out}


def case_stream() -> dict:
    w = synth.workload("stream_frame")
    frames, total = [], None
    for k in range(STREAM_FRAMES):
        s = synth.stream_frame(k)
        v = oracle.correlate(s)
        total = v if total is None else total + v
        frames.append({"k": k, "input_sha256": sha(s), "vis_sha256": vis_digest(v)})
    return {"N": w.N, "F": w.F, "T": w.T, "recipe": w.kind, "seed": w.seed,
            "frames": frames, "sum_vis_sha256": vis_digest(total)}


CASES = {
    "tiny": lambda: case_workload("tiny"),
    "pathfinder": lambda: case_workload("pathfinder"),
    "full_array": lambda: case_workload("full_array"),
    "precision_subset": case_precision,
    "batch": case_batch,
    "stream": case_stream,
}


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--only", choices=sorted(CASES), action="append")
    args = ap.parse_args()
    data = {"format": "sha256 of int32 [F][N(N+1)/2][2] little-endian, C order", "cases": {}}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in args.only or list(CASES):
        t0 = time.time()
        data["cases"][name] = CASES[name]()
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()
