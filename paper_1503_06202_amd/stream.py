"""Streaming request loop: continuous batching of integration frames.

Frames of 4+4-bit samples arrive over time (a Poisson process in the
benchmark).  Each frame belongs to a stream, i.e. an instrument whose
visibilities integrate frame after frame (Sec. IV-C, "Full Correlation": the
correlation matrix is integrated, by default over 2^23 samples, then dumped).
The loop keeps one accumulator per stream resident on the GPU and dumps it
every ``dump_every`` frames.

Continuous batching: a frame is admitted as soon as a slot (device memory for
one in-flight frame) is free; whenever fewer than ``max_inflight`` launches
are on the GPU, the admitted frames not yet launched (up to the launcher's
``max_batch``) go out in one batched launch, so frames that arrive while
others run are picked up at the next launch instead of waiting for a drained
queue.  Two launches are in flight by default: the GPU launcher queues them
on one HIP stream, so the second starts on the device as soon as the first
ends, while the host forms the next batch.  It can also spread launches over
several HIP streams (``queues``), where a launch fills the compute units the
previous one leaves idle as it drains; on full-size frames two concurrent
batched kernels served fewer frames per second than two queued launches, and
with a longer p99.  Frames of one stream may share a launch, and launches on
any HIP stream add into the same accumulator: the batched kernels add with
exact int32 atomics, whose order does not matter.  Latency is measured from a
frame's arrival to the completion of the launch that carried it.

The loop talks to a launcher (``launch``, ``ready``, ``dump``); the GPU
launcher below drives ``libxeng.so`` through batched plans, one set per HIP
stream, optionally replaying captured HIP graphs.  An integration can be
checkpointed (``GpuLauncher.checkpoint`` with the loop's per-stream frame
counts) and resumed in another launcher (``restore``, ``RequestLoop.run(...,
since_dump=...)``) with the same result as an uninterrupted run.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import math
import os
import time
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np


class Markers:
    """roctx ranges (ROCm's marker API, which ``rocprofv3 --marker-trace``
    records beside the kernels), or no-ops where no roctx library loads.
    The request loop opens one range per run, per launch and per dump."""

    def __init__(self):
        self._push = self._pop = None
        lib_dir = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
        for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"):
            for path in (os.path.join(lib_dir, name), name):
                try:
                    lib = ctypes.CDLL(path)
                except OSError:
                    continue
                lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                lib.roctxRangePushA.restype = ctypes.c_int
                lib.roctxRangePop.argtypes = []
                lib.roctxRangePop.restype = ctypes.c_int
                self._push, self._pop = lib.roctxRangePushA, lib.roctxRangePop
                self.library = path
                return
        self.library = None

    def push(self, message: str) -> None:
        if self._push is not None:
            self._push(message.encode())

    def pop(self) -> None:
        if self._pop is not None:
            self._pop()


_markers: Optional[Markers] = None


def default_markers() -> Markers:
    global _markers
    if _markers is None:
        _markers = Markers()
    return _markers


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

    def __init__(self, launcher, max_inflight: Optional[int] = None, dump_every: int = 256,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, markers=None):
        if max_inflight is None:
            max_inflight = 2  # the next launch waits on the device, not on the host
        if launcher.slots < 1 or max_inflight < 1 or dump_every < 1:
            raise ValueError("slots, max_inflight and dump_every must be >= 1")
        self.launcher = launcher
        self.max_inflight = max_inflight
        self.max_batch = getattr(launcher, "max_batch", launcher.slots)
        self.dump_every = dump_every
        self.clock = clock
        self.sleep = sleep
        self.markers = markers if markers is not None else default_markers()

    def run(self, frames: Sequence[Frame], since_dump: Optional[Dict[int, int]] = None) -> Report:
        """Serve ``frames``; ``since_dump`` resumes an integration (frames already
        integrated per stream since the last dump, e.g. from a checkpoint)."""
        frames = sorted(frames, key=lambda f: f.arrival)
        slots = self.launcher.slots
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        arriving: Deque[Frame] = collections.deque(frames)
        waiting: Deque[Frame] = collections.deque()     # arrived, no slot yet
        admitted: Deque[Frame] = collections.deque()    # holds a slot, not launched
        inflight: List[tuple] = []                      # (token, frames), launch order
        used = 0
        counts: Dict[int, int] = collections.defaultdict(int, since_dump or {})
        dumps: List[Any] = []
        batch_sizes: List[int] = []
        finished: List[Frame] = []
        mk = self.markers
        mk.push(f"request loop: {len(frames)} frames")
        while arriving or waiting or admitted or inflight:
            t = now()
            while arriving and arriving[0].arrival <= t:
                waiting.append(arriving.popleft())
            # completions free their slots (launches on different HIP streams
            # may complete out of order)
            if inflight:
                still = []
                for token, fs in inflight:
                    if self.launcher.ready(token):
                        td = now()
                        for f in fs:
                            f.done = td
                        finished.extend(fs)
                        used -= len(fs)
                    else:
                        still.append((token, fs))
                inflight = still
            while waiting and used < slots:
                f = waiting.popleft()
                f.admitted = t
                admitted.append(f)
                used += 1
            if admitted and len(inflight) < self.max_inflight:
                batch = [admitted.popleft() for _ in range(min(len(admitted), self.max_batch))]
                tl = now()
                for f in batch:
                    f.launched = tl
                    f.batch = len(batch)
                mk.push(f"launch: {len(batch)} frames")
                token = self.launcher.launch(batch)
                mk.pop()
                inflight.append((token, batch))
                batch_sizes.append(len(batch))
                for f in batch:
                    counts[f.stream] += 1
                # a dump is ordered after every launch so far, so it holds every
                # frame of the stream launched since the previous dump (its
                # count is kept)
                for st in sorted({f.stream for f in batch}):
                    if counts[st] >= self.dump_every:
                        mk.push(f"dump: stream {st}, {counts[st]} frames")
                        dumps.append((st, counts[st], self.launcher.dump(st)))
                        mk.pop()
                        counts[st] = 0
                continue
            blocked = bool(admitted) and len(inflight) >= self.max_inflight
            if blocked or (not (waiting and used < slots) and not admitted):
                # idle until the next arrival or completion (admitted frames
                # waiting for a launch slot wait for a completion too)
                if inflight:
                    self.launcher.poll_wait(inflight[0][0])
                elif arriving:
                    dt = arriving[0].arrival - now()
                    if dt > 0:
                        self.sleep(min(dt, 0.001))
        wall = now()
        mk.pop()
        lat = np.array([f.latency * 1e3 for f in finished])
        rep = Report(len(finished), wall, lat, batch_sizes, dumps)
        rep.pending = dict(counts)  # frames integrated since the last dump, per stream
        return rep


def slots_from_memory(frame_bytes: int, fraction: float = 0.5, cap: int = 128,
                      device=None) -> int:
    """Slots (frames admitted at once) that ``fraction`` of the free device
    memory holds, at most ``cap``."""
    import torch

    free, _ = torch.cuda.mem_get_info(device)
    return int(max(1, min(cap, (free * fraction) // max(1, frame_bytes))))


class GpuLauncher:
    """Runs batches of frames of one shape through ``libxeng.so``.

    Launches go to an idle one of ``queues`` HIP streams (default priority),
    else to the next in turn.  With one HIP stream (the default) launches run
    one after another on the device, the next queued behind the current one;
    with several, a launch starts filling the compute units while the
    previous one drains (measured slower on full-size frames than two
    launches in a row on one stream).
    Each HIP stream has its own batched plans, one per batch size k =
    1..``max_batch`` (k identical instances (N, F, T)), because a plan's calls
    must not overlap on the device (calls on one HIP stream run in order); a
    plan's automatic time slices are chosen for k
    frames' worth of tiles, so that a lone frame spreads over the whole GPU
    as well as a full batch does.  Every stream's accumulator lives on the
    GPU; frames add into it (shared, atomic) from any HIP stream.  ``dump``
    is ordered after the last launch on every HIP stream, copies the
    accumulator into one of ``dump_buffers`` pinned host buffers allocated up
    front (in turn: a dump's buffer is reused ``dump_buffers`` dumps later),
    and clears it; the next launches wait for the clear.
    ``slots`` bounds the frames admitted at once (default: what half of the
    free device memory holds, at most 128).  ``tune_slices`` times the time
    slices per tile of every batch size on real frames and keeps the fastest
    exact choice (the automatic count is a cost model).
    """

    def __init__(self, N: int, F: int, T: int, slots: Optional[int] = None, streams: int = 1,
                 form: str = "i8", graph: bool = True, device=None, max_batch: int = 8,
                 queues: int = 1, dump_buffers: int = 4):
        import torch

        from .engine import vis_shape

        self.torch = torch
        self.N, self.F, self.T = N, F, T
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        frame_bytes = N * F * T
        self.slots = int(slots) if slots else slots_from_memory(frame_bytes, device=self.device)
        self.max_batch = max(1, min(max_batch, self.slots))
        self.graph = graph
        self.form = form
        self.queues = max(1, int(queues))
        self.hip_streams = [torch.cuda.Stream(self.device) for _ in range(self.queues)]
        self.plans = [{k: self._plan(k, 0) for k in range(1, self.max_batch + 1)}
                      for _ in range(self.queues)]
        self.split_t = {k: 0 for k in range(1, self.max_batch + 1)}  # 0: the library's choice
        self.split_ms: Dict[int, Dict[int, float]] = {}
        shape = vis_shape(N, F)
        self.acc = [torch.zeros(shape, dtype=torch.int32, device=self.device)
                    for _ in range(streams)]
        self.dump_bufs = [torch.empty(shape, dtype=torch.int32, pin_memory=True)
                          for _ in range(max(1, dump_buffers))]
        self.dump_events = [None] * len(self.dump_bufs)
        self._next_dump = 0
        self._next_q = 0
        self._last = [None] * self.queues   # last launch event per HIP stream
        self._cleared = None                # event after the latest accumulator clear
        # the accumulators were written on the current stream
        for s in self.hip_streams:
            s.wait_stream(torch.cuda.current_stream(self.device))

    def _pick_queue(self) -> int:
        """An idle HIP stream (its last launch has completed), else the next in turn."""
        for i in range(self.queues):
            q = (self._next_q + i) % self.queues
            if self._last[q] is None or self._last[q].query():
                return q
        return self._next_q

    def launch(self, frames: List[Frame]):
        q = self._pick_queue()
        self._next_q = (q + 1) % self.queues
        return self._launch_on(q, frames)

    def _launch_on(self, q: int, frames: List[Frame]):
        torch = self.torch
        s = self.hip_streams[q]
        if self._cleared is not None:
            s.wait_event(self._cleared)
        samples = [f.samples for f in frames]
        vis = [self.acc[f.stream] for f in frames]
        self.plans[q][len(frames)].correlate(samples, vis, stream=s, graph=self.graph)
        ev = torch.cuda.Event()
        ev.record(s)
        self._last[q] = ev
        return ev

    def _plan(self, k: int, split: int):
        from .engine import BatchPlan

        return BatchPlan([(self.N, self.F, self.T)] * k, form=self.form, accumulate=True,
                         shared_vis=True, split_t=[split] * k)

    def tune_slices(self, samples, candidates: Sequence[int] = (0, 2, 3, 4),
                    reps: int = 5) -> Dict[int, int]:
        """Time slices per tile for every batch size k: each candidate (0: the
        library's automatic count) is timed as this launcher runs it (a
        batched plan of k frames adding into one accumulator, graph-replayed
        on the first HIP stream) on ``samples``; the fastest whose result is
        bit-identical to the automatic count's replaces the plans of size k on
        every HIP stream.  The launcher's accumulators are not touched."""
        torch = self.torch
        s = self.hip_streams[0]
        scratch = torch.zeros_like(self.acc[0])
        # the clocks of an idle GPU ramp up under load: run the largest batch
        # for a while before timing anything
        big = self.plans[0][self.max_batch]
        frames = [samples[i % len(samples)] for i in range(self.max_batch)]
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.3:
            with torch.cuda.stream(s):
                scratch.zero_()  # keep the sums far from the int32 range
            big.correlate(frames, [scratch] * self.max_batch, stream=s, graph=self.graph)
            torch.cuda.synchronize(self.device)
        for k in range(1, self.max_batch + 1):
            frames = [samples[i % len(samples)] for i in range(k)]
            ref, times = None, {}
            n = max(reps, -(-reps * 4 // k))  # at least about 4 reps' worth of frames
            for split in dict.fromkeys([0] + [int(c) for c in candidates]):
                plan = self._plan(k, split)
                with torch.cuda.stream(s):
                    scratch.zero_()
                    plan.correlate(frames, [scratch] * k, stream=s, graph=self.graph)
                    got = scratch.clone()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(s)
                    for _ in range(n):
                        plan.correlate(frames, [scratch] * k, stream=s, graph=self.graph)
                    e1.record(s)
                e1.synchronize()
                if ref is None:
                    ref = got
                if torch.equal(got, ref):  # never keep a count that changes a bit
                    times[split] = e0.elapsed_time(e1) / n
                plan.close()
            best = min(times, key=times.get)
            self.split_ms[k] = times
            if best != self.split_t[k]:
                for q in range(self.queues):
                    self.plans[q][k].close()
                    self.plans[q][k] = self._plan(k, best)
                self.split_t[k] = best
        torch.cuda.synchronize(self.device)
        return dict(self.split_t)

    def warm(self, samples) -> None:
        """Run every plan once (capturing its graph) on ``samples``, then clear
        the accumulators, so that no launch in a timed run pays for a capture."""
        for q in range(self.queues):
            for k in range(1, self.max_batch + 1):
                frames = [Frame(-1, 0, samples[i % len(samples)], 0.0) for i in range(k)]
                self._launch_on(q, frames)
        self.torch.cuda.synchronize(self.device)
        for a in self.acc:
            a.zero_()
        self.torch.cuda.synchronize(self.device)

    def ready(self, token) -> bool:
        return token.query()

    def poll_wait(self, token) -> None:
        """Called while idle with work in flight: spin (completions take well under 1 ms)."""

    def _after_all(self):
        """A HIP stream ordered after the last launch on every HIP stream."""
        s = self.hip_streams[0]
        for q in range(1, self.queues):
            if self._last[q] is not None:
                s.wait_event(self._last[q])
        return s

    def dump(self, stream: int):
        torch = self.torch
        s = self._after_all()
        b = self._next_dump
        self._next_dump = (b + 1) % len(self.dump_bufs)
        if self.dump_events[b] is not None:
            self.dump_events[b].synchronize()  # its previous copy has landed
        host = self.dump_bufs[b]
        with torch.cuda.stream(s):
            host.copy_(self.acc[stream], non_blocking=True)
            self.acc[stream].zero_()
        ev = torch.cuda.Event()
        ev.record(s)
        self.dump_events[b] = ev
        self._cleared = ev
        return (stream, host, ev)

    def checkpoint(self) -> List[Any]:
        """Host copies of every accumulator, after all launched work (blocks)."""
        s = self._after_all()
        s.synchronize()
        return [a.cpu().clone() for a in self.acc]

    def restore(self, state: Sequence[Any]) -> None:
        """Load accumulators saved by ``checkpoint`` (into this launcher)."""
        torch = self.torch
        if len(state) != len(self.acc):
            raise ValueError("checkpoint holds a different number of streams")
        s = self._after_all()
        with torch.cuda.stream(s):
            for a, h in zip(self.acc, state):
                a.copy_(torch.as_tensor(h).to(self.device, non_blocking=False))
        ev = torch.cuda.Event()
        ev.record(s)
        self._cleared = ev
        s.synchronize()

    def close(self) -> None:
        for q in self.plans:
            for p in q.values():
                p.close()
