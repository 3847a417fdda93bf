"""Autotuners: tile shape and time slices of a plain plan, and time slices
per instance shape of a batched plan.

Plain form (``tune_plain``): for one frame shape (N, F, T) the tuner times
every kernel shape the library has on seeded synthetic frames of that shape:
the channel kernel (kernel 5 of ``xeng_plan_set_tuning``; int8, N <= 256),
128 x 128 tiles with split or common wave roles in diagonal tiles (kernel 3
or 4) and 128 x 256 tiles (kernel 2), each with the automatic time slices and
with 1, 2 and 4 slices.  It rejects any
candidate whose output is not bit-identical to the first candidate's, keeps
the fastest, and caches it as JSON keyed by (arch, form, N, F, T).

Batched form (``tune``):

A batched plan launches one persistent kernel over the tiles of every
instance.  Splitting an instance's integration into several time slices gives
the scheduler more, smaller work items (better load balance across uneven N),
at the price of exact integer atomic adds into vis and a clear beforehand.  For
every distinct shape (N, F, T) of a batch, the tuner times candidate splits on
a batch that holds as many copies of that shape as the real batch does, on
seeded synthetic frames, rejects any candidate whose output is not bit-identical
to the unsplit one, and keeps the fastest.  Results are cached as JSON keyed by
(arch, form, N, F, T).
"""
from __future__ import annotations

import json
import os
from collections import Counter
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

CANDIDATES = (1, 2, 4, 8)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "xeng_tune.json")


def _key(arch: str, form: str, N: int, F: int, T: int) -> str:
    return f"{arch}/{form}/{N}x{F}x{T}"


def _arch() -> str:
    import torch

    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", "gpu").split(":")[0]


def load_cache(path: str) -> Dict[str, dict]:
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def save_cache(path: str, cache: Dict[str, dict]) -> None:
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


PLAIN_KERNELS = (5, 3, 4, 2)  # channel kernel, 128x128 split diagonal, 128x128 common, 128x256
PLAIN_SPLITS = (0, 1, 2, 4)   # 0: automatic


def _time_plain(shape, form: str, kernel: int, split: int, frame, reps: int):
    import torch

    from .engine import Plan

    N, F, T = shape
    with Plan(N, F, T, form=form, split_t=split, kernel=kernel) as p:
        out = p.correlate(frame)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            e0.record()
            p.correlate(frame, out)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2], out


def tune_plain(N: int, F: int, T: int, form: str = "i8", kernels: Iterable[int] = PLAIN_KERNELS,
               splits: Iterable[int] = PLAIN_SPLITS, reps: int = 5,
               cache_path: Optional[str] = DEFAULT_CACHE, seed: int = 4321, frame=None,
               log=None, times: Optional[Dict[str, float]] = None) -> Tuple[int, int]:
    """(kernel, split_t) for ``Plan.set_tuning`` on frames of this shape.

    ``frame`` (optional): a device frame of the shape to time on, instead of a
    freshly generated one.  ``times`` (optional): filled with the median
    milliseconds of every exact candidate, keyed "kernel/split".
    """
    import torch

    import synth

    key = "plain/" + _key(_arch(), form, N, F, T)
    cache = load_cache(cache_path) if cache_path else {}
    if key in cache:
        if times is not None:
            times.update(cache[key].get("ms", {}))
        return int(cache[key]["kernel"]), int(cache[key]["split_t"])
    if frame is None:
        frame = torch.from_numpy(synth.gen_frame(N, F, T, seed, "gauss",
                                                 stream_key=(0x7F, N, T))).cuda()
    results, ref = {}, None
    for kernel in kernels:
        if kernel == 2 and N % 16:
            continue  # 128 x 256 tiles need 16-aligned inputs
        if kernel == 5 and (N > 256 or form != "i8"):
            continue  # the channel kernel: int8, at most 256 inputs
        for split in splits:
            if split > max(1, T // 64):
                continue
            ms, out = _time_plain((N, F, T), form, kernel, split, frame, reps)
            if ref is None:
                ref = out
            elif not torch.equal(out, ref):  # never keep a candidate that changes a bit
                if log:
                    log(f"tune: {key} kernel {kernel} split {split} rejected (not bit-exact)")
                continue
            results[(kernel, split)] = ms
    choice = min(results, key=results.get)
    cache[key] = {"kernel": choice[0], "split_t": choice[1],
                  "ms": {f"{k}/{s}": v for (k, s), v in sorted(results.items())}}
    if times is not None:
        times.update(cache[key]["ms"])
    if log:
        log(f"tune: {key}: " + ", ".join(f"kernel {k} split {s}: {v:.3f} ms"
                                          for (k, s), v in sorted(results.items())) +
            f" -> kernel {choice[0]} split {choice[1]}")
    if cache_path:
        save_cache(cache_path, cache)
    return choice


def _time_batch(shape: Tuple[int, int, int], copies: int, split: int, form: str, frames,
                reps: int) -> Tuple[float, list]:
    import torch

    from .engine import BatchPlan, vis_shape

    N, F, T = shape
    vis = [torch.empty(vis_shape(N, F), dtype=torch.int32, device=frames[0].device)
           for _ in range(copies)]
    with BatchPlan([shape] * copies, form=form, split_t=[split] * copies) as bp:
        bp.correlate(frames, vis, graph=True)  # warm-up, captures the graph
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            e0.record()
            bp.correlate(frames, vis, graph=True)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2], vis


def tune(instances: Sequence[Tuple[int, int, int]], form: str = "i8",
         candidates: Iterable[int] = CANDIDATES, reps: int = 3,
         cache_path: Optional[str] = DEFAULT_CACHE, seed: int = 1234,
         frames: Optional[Sequence] = None, log=None) -> List[int]:
    """split_t for every instance of the batch (same order).

    ``frames`` (optional): the batch's own device frames, used for timing
    instead of freshly generated ones.
    """
    import torch

    import synth

    arch = _arch()
    cache = load_cache(cache_path) if cache_path else {}
    counts = Counter(tuple(map(int, s)) for s in instances)
    best: Dict[Tuple[int, int, int], int] = {}
    for shape, copies in sorted(counts.items()):
        key = _key(arch, form, *shape)
        if key in cache and cache[key].get("copies") == copies:
            best[shape] = int(cache[key]["split_t"])
            continue
        N, F, T = shape
        if frames is not None:
            own = [fr for s, fr in zip(instances, frames) if tuple(map(int, s)) == shape]
        else:
            own = [torch.from_numpy(synth.gen_frame(N, F, T, seed + k, "gauss",
                                                    stream_key=(0x7E, N, T))).cuda()
                   for k in range(copies)]
        ref_ms, ref = _time_batch(shape, copies, 1, form, own, reps)
        results = {1: ref_ms}
        for split in candidates:
            if split == 1 or split > max(1, T // 64):
                continue
            ms, out = _time_batch(shape, copies, split, form, own, reps)
            exact = all(torch.equal(a, b) for a, b in zip(out, ref))
            if not exact:  # never keep a candidate that changes a single bit
                if log:
                    log(f"tune: {key} split {split} rejected (not bit-exact)")
                continue
            results[split] = ms
        choice = min(results, key=results.get)
        best[shape] = choice
        cache[key] = {"split_t": choice, "copies": copies,
                      "ms": {str(k): v for k, v in results.items()}}
        if log:
            log(f"tune: {key} x{copies}: " +
                ", ".join(f"split {k}: {v:.3f} ms" for k, v in sorted(results.items())) +
                f" -> {choice}")
        del own, ref
    if cache_path:
        save_cache(cache_path, cache)
    return [best[tuple(map(int, s))] for s in instances]
