"""Streaming request loop: continuous batching of integration frames.

Frames of 4+4-bit samples arrive over time (a Poisson process in the
benchmark).  Each frame belongs to a stream, i.e. an instrument whose
visibilities integrate frame after frame (Sec. IV-C, "Full Correlation": the
correlation matrix is integrated, by default over 2^23 samples, then dumped).
The loop keeps one accumulator per stream resident on the GPU and dumps it
every ``dump_every`` frames.

Continuous batching: a frame is admitted as soon as a slot (device memory for
one in-flight frame) is free; whenever fewer than ``max_inflight`` launches
are on the GPU, every admitted frame not yet launched goes out in one batched
launch, so frames that arrive while others run are picked up at the next
launch instead of waiting for a drained queue.  Frames of one stream may share
a launch: the batched kernels add into the shared accumulator with exact
int32 atomics.  Latency is measured from a frame's arrival to the completion
of the launch that carried it.

The loop talks to a launcher (``launch``, ``ready``, ``dump``); the GPU
launcher below drives ``libxeng.so`` through a batched plan over the slots,
optionally replaying a captured HIP graph.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Frame:
    fid: int
    stream: int
    samples: Any          # what the launcher correlates (a device tensor for the GPU)
    arrival: float        # seconds after the start of the run
    admitted: float = math.nan
    launched: float = math.nan
    done: float = math.nan
    batch: int = 0        # frames in the launch that carried it

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class Report:
    frames: int
    wall_s: float
    latencies_ms: np.ndarray
    batch_sizes: List[int]
    dumps: List[Any]          # (stream, frames in the dump, launcher's dump payload)
    pending: Dict[int, int] = dataclasses.field(default_factory=dict)

    @property
    def frames_per_s(self) -> float:
        return self.frames / self.wall_s if self.wall_s > 0 else math.nan

    def pct(self, q: float) -> float:
        return float(np.percentile(self.latencies_ms, q)) if len(self.latencies_ms) else math.nan

    def summary(self) -> Dict[str, float]:
        return {"frames": self.frames, "wall_s": self.wall_s, "frames_per_s": self.frames_per_s,
                "p50_ms": self.pct(50), "p99_ms": self.pct(99),
                "max_ms": float(self.latencies_ms.max()) if len(self.latencies_ms) else math.nan,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                "launches": len(self.batch_sizes), "dumps": len(self.dumps)}


def poisson_arrivals(n: int, rate_hz: float, seed: int) -> np.ndarray:
    """Arrival times (s) of n frames of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    if not math.isfinite(rate_hz) or rate_hz <= 0:
        return np.zeros(n)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n)) - 0.0


class RequestLoop:
    """Admission, continuous batching, completion and dumps over a launcher."""

    def __init__(self, launcher, max_inflight: int = 2, dump_every: int = 256,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        if launcher.slots < 1 or max_inflight < 1 or dump_every < 1:
            raise ValueError("slots, max_inflight and dump_every must be >= 1")
        self.launcher = launcher
        self.max_inflight = max_inflight
        self.dump_every = dump_every
        self.clock = clock
        self.sleep = sleep

    def run(self, frames: Sequence[Frame]) -> Report:
        frames = sorted(frames, key=lambda f: f.arrival)
        slots = self.launcher.slots
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        arriving: Deque[Frame] = collections.deque(frames)
        waiting: Deque[Frame] = collections.deque()     # arrived, no slot yet
        admitted: Deque[Frame] = collections.deque()    # holds a slot, not launched
        inflight: Deque[tuple] = collections.deque()    # (token, frames)
        used = 0
        since_dump: Dict[int, int] = collections.defaultdict(int)
        dumps: List[Any] = []
        batch_sizes: List[int] = []
        finished: List[Frame] = []
        while arriving or waiting or admitted or inflight:
            t = now()
            while arriving and arriving[0].arrival <= t:
                waiting.append(arriving.popleft())
            # completions free their slots
            while inflight and self.launcher.ready(inflight[0][0]):
                _, fs = inflight.popleft()
                td = now()
                for f in fs:
                    f.done = td
                finished.extend(fs)
                used -= len(fs)
            while waiting and used < slots:
                f = waiting.popleft()
                f.admitted = t
                admitted.append(f)
                used += 1
            if admitted and len(inflight) < self.max_inflight:
                batch = list(admitted)
                admitted.clear()
                tl = now()
                for f in batch:
                    f.launched = tl
                    f.batch = len(batch)
                token = self.launcher.launch(batch)
                inflight.append((token, batch))
                batch_sizes.append(len(batch))
                for f in batch:
                    since_dump[f.stream] += 1
                # a dump is ordered after this launch, so it holds every frame of
                # the stream launched since the previous dump (its count is kept)
                for st in sorted({f.stream for f in batch}):
                    if since_dump[st] >= self.dump_every:
                        dumps.append((st, since_dump[st], self.launcher.dump(st)))
                        since_dump[st] = 0
                continue
            if not (waiting and used < slots) and not admitted:
                # idle until the next arrival or completion
                if inflight:
                    self.launcher.poll_wait(inflight[0][0])
                elif arriving:
                    dt = arriving[0].arrival - now()
                    if dt > 0:
                        self.sleep(min(dt, 0.001))
        wall = now()
        lat = np.array([f.latency * 1e3 for f in finished])
        rep = Report(len(finished), wall, lat, batch_sizes, dumps)
        rep.pending = dict(since_dump)  # frames integrated since the last dump, per stream
        return rep


class GpuLauncher:
    """Runs batches of frames of one shape through ``libxeng.so``.

    There is one batched plan per batch size k = 1..``slots`` (k identical
    instances (N, F, T)); a launch of k frames uses the plan of size k, whose
    automatic time slices are chosen for k frames' worth of tiles, so that a
    lone frame spreads over the whole GPU as well as a full batch does.
    Every stream's accumulator lives on the GPU; frames add into it (shared,
    atomic) and ``dump`` enqueues an asynchronous copy to pinned host memory
    followed by a clear, all ordered on the launch stream.
    """

    def __init__(self, N: int, F: int, T: int, slots: int, streams: int = 1, form: str = "i8",
                 graph: bool = True, device=None):
        import torch

        from .engine import BatchPlan, vis_shape

        self.torch = torch
        self.N, self.F, self.T = N, F, T
        self.slots = slots
        self.graph = graph
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        self.plans = {k: BatchPlan([(N, F, T)] * k, form=form, accumulate=True, shared_vis=True)
                      for k in range(1, slots + 1)}
        self.acc = [torch.zeros(vis_shape(N, F), dtype=torch.int32, device=self.device)
                    for _ in range(streams)]

    def launch(self, frames: List[Frame]):
        torch = self.torch
        plan = self.plans[len(frames)]
        samples = [f.samples for f in frames]
        vis = [self.acc[f.stream] for f in frames]
        plan.correlate(samples, vis, stream=self.stream, graph=self.graph)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def warm(self, samples) -> None:
        """Run every plan once (capturing its graph) on ``samples``, then clear
        the accumulators, so that no launch in a timed run pays for a capture."""
        for k in range(1, self.slots + 1):
            frames = [Frame(-1, 0, samples[i % len(samples)], 0.0) for i in range(k)]
            self.launch(frames)
        for a in self.acc:
            a.zero_()
        self.torch.cuda.synchronize(self.device)

    def ready(self, token) -> bool:
        return token.query()

    def poll_wait(self, token) -> None:
        """Called while idle with work in flight: spin (completions take well under 1 ms)."""

    def dump(self, stream: int):
        torch = self.torch
        host = torch.empty(self.acc[stream].shape, dtype=torch.int32, pin_memory=True)
        host.copy_(self.acc[stream], non_blocking=True)
        self.acc[stream].zero_()
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return (stream, host, ev)

    def close(self) -> None:
        for p in self.plans.values():
            p.close()
