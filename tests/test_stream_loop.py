"""The streaming request loop's admission, batching and dump logic, on the CPU
with a fake launcher that completes launches after a fixed service time on a
virtual clock and integrates frames with the oracle."""
import collections

import numpy as np
import pytest

import oracle
from paper_1503_06202_amd.stream import Frame, RequestLoop, poisson_arrivals


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeLauncher:
    def __init__(self, clock, slots, service_s, per_frame_s=0.0, streams=1):
        self.clock, self.slots = clock, slots
        self.service_s, self.per_frame_s = service_s, per_frame_s
        self.acc = collections.defaultdict(lambda: 0)
        self.in_device = 0
        self.max_in_device = 0
        self.launches = []

    def launch(self, frames):
        done_at = self.clock() + self.service_s + self.per_frame_s * len(frames)
        if self.launches and self.launches[-1] > self.clock():
            done_at = self.launches[-1] + self.service_s + self.per_frame_s * len(frames)
        self.launches.append(done_at)
        for f in frames:
            self.acc[f.stream] = self.acc[f.stream] + oracle.correlate(f.samples)
        self.in_device += len(frames)
        self.max_in_device = max(self.max_in_device, self.in_device)
        return (done_at, len(frames))

    def ready(self, token):
        ok = self.clock() >= token[0]
        if ok:
            self.in_device -= token[1]
            token_done = True  # noqa: F841
        return ok

    def poll_wait(self, token):
        self.clock.t = max(self.clock.t, token[0])

    def dump(self, stream):
        out = self.acc[stream]
        self.acc[stream] = 0
        return out

    def checkpoint(self):
        return dict(self.acc)

    def restore(self, state):
        self.acc = collections.defaultdict(lambda: 0, state)


def frames_for(n, streams, rate, seed=0, N=6, F=2, T=16):
    rng = np.random.default_rng(seed)
    arr = poisson_arrivals(n, rate, seed)
    return [Frame(k, k % streams, rng.integers(0, 256, (T, F, N), dtype=np.uint8), float(arr[k]))
            for k in range(n)]


def test_every_frame_completes_with_latency_at_least_service():
    clk = VClock()
    la = FakeLauncher(clk, slots=4, service_s=0.002)
    fr = frames_for(60, 1, rate=300.0)
    rep = RequestLoop(la, max_inflight=2, dump_every=1000, clock=clk, sleep=clk.sleep).run(fr)
    assert rep.frames == 60
    assert (rep.latencies_ms >= 2.0 - 1e-9).all()
    assert la.max_in_device <= 4


def test_overload_batches_and_respects_slots():
    # all frames at t = 0: the loop must batch up to `slots` and never exceed it
    clk = VClock()
    la = FakeLauncher(clk, slots=5, service_s=0.001)
    fr = frames_for(40, 2, rate=float("inf"))
    rep = RequestLoop(la, max_inflight=2, dump_every=1000, clock=clk, sleep=clk.sleep).run(fr)
    assert rep.frames == 40
    assert max(rep.batch_sizes) <= 5 and sum(rep.batch_sizes) == 40
    assert max(rep.batch_sizes) > 1
    assert la.max_in_device <= 5


def test_continuous_batching_picks_up_arrivals_during_flight():
    # slow service, frequent arrivals: later launches carry several frames
    clk = VClock()
    la = FakeLauncher(clk, slots=8, service_s=0.010)
    fr = frames_for(50, 1, rate=1000.0)
    rep = RequestLoop(la, max_inflight=1, dump_every=1000, clock=clk, sleep=clk.sleep).run(fr)
    assert rep.frames == 50
    assert np.mean(rep.batch_sizes[1:]) > 3


@pytest.mark.parametrize("streams,dump_every", [(1, 7), (3, 5)])
def test_dumps_plus_pending_equal_sum_of_frames(streams, dump_every):
    clk = VClock()
    la = FakeLauncher(clk, slots=3, service_s=0.001, streams=streams)
    fr = frames_for(45, streams, rate=2000.0, seed=3)
    rep = RequestLoop(la, max_inflight=2, dump_every=dump_every, clock=clk, sleep=clk.sleep).run(fr)
    for st in range(streams):
        want = sum(oracle.correlate(f.samples) for f in fr if f.stream == st)
        dumped = [d for s, n, d in rep.dumps if s == st]
        counts = [n for s, n, d in rep.dumps if s == st]
        assert all(n >= dump_every for n in counts)
        total = sum(dumped) + la.acc[st]
        assert np.array_equal(total, want)
        assert sum(counts) + rep.pending.get(st, 0) == sum(1 for f in fr if f.stream == st)


def test_rejects_bad_configuration():
    clk = VClock()
    with pytest.raises(ValueError):
        RequestLoop(FakeLauncher(clk, slots=0, service_s=0.001))
    with pytest.raises(ValueError):
        RequestLoop(FakeLauncher(clk, slots=1, service_s=0.001), max_inflight=0)


def test_checkpoint_and_resume_dump_like_an_uninterrupted_run():
    # the loop's per-stream counts since the last dump travel with the
    # launcher's accumulators: a resumed run dumps at the same frames and the
    # same sums as one that was never interrupted
    fr = frames_for(23, 2, 300.0, seed=4)

    def run(frs, la, since=None):
        clk = la.clock
        return RequestLoop(la, max_inflight=2, dump_every=5, clock=clk, sleep=clk.sleep).run(
            frs, since_dump=since)

    clk = VClock()
    la = FakeLauncher(clk, slots=3, service_s=0.002)
    whole = run(fr, la)
    clk1 = VClock()
    la1 = FakeLauncher(clk1, slots=3, service_s=0.002)
    first = run(fr[:11], la1)
    state, since = la1.checkpoint(), dict(first.pending)
    clk2 = VClock()
    la2 = FakeLauncher(clk2, slots=3, service_s=0.002)
    la2.restore(state)
    for f in fr[11:]:
        f.arrival -= fr[11].arrival
    second = run(fr[11:], la2, since)
    got = first.dumps + second.dumps
    assert [(s, c) for s, c, _ in got] == [(s, c) for s, c, _ in whole.dumps]
    for (_, _, a), (_, _, b) in zip(got, whole.dumps):
        assert np.array_equal(a, b)
    assert second.pending == whole.pending
    for st in (0, 1):
        assert np.array_equal(np.asarray(la2.acc[st]), np.asarray(la.acc[st]))


def single_server_latencies(arrivals, service, max_inflight, max_batch):
    """Latency of every frame (arrival order) under the loop's policy, as a
    plain event recursion: whenever fewer than ``max_inflight`` launches are
    outstanding, every waiting frame (at most ``max_batch``) goes out in one
    launch; launches are served one after another, a launch of k frames
    taking service(k) seconds."""
    n, lat = len(arrivals), [0.0] * len(arrivals)
    waiting, i, t, free, outstanding = collections.deque(), 0, 0.0, 0.0, []
    while i < n or waiting:
        outstanding = [c for c in outstanding if c > t]
        while i < n and arrivals[i] <= t:
            waiting.append(i)
            i += 1
        if waiting and len(outstanding) < max_inflight:
            batch = [waiting.popleft() for _ in range(min(len(waiting), max_batch))]
            done = max(t, free) + service(len(batch))
            free = done
            outstanding.append(done)
            for k in batch:
                lat[k] = done - arrivals[k]
            continue
        t = min(outstanding + ([arrivals[i]] if i < n else []))
    return np.array(lat)


class ExactLauncher(FakeLauncher):
    """Waits until the next completion or arrival, whichever comes first, so
    that the loop sees every event at its exact time."""

    def __init__(self, clock, arrivals, max_batch, **kw):
        super().__init__(clock, **kw)
        self.arrivals = np.sort(np.asarray(arrivals))
        self.max_batch = max_batch  # the loop's batch cap, as GpuLauncher sets it

    def poll_wait(self, token):
        k = int(np.searchsorted(self.arrivals, self.clock.t, side="right"))
        nxt = self.arrivals[k] if k < len(self.arrivals) else float("inf")
        self.clock.t = max(self.clock.t, min(token[0], nxt))


@pytest.mark.parametrize("max_inflight", [1, 2])
def test_loop_matches_single_server_model(max_inflight):
    # launch times close to the GPU's for the stream frames (a fixed 0.07 ms
    # plus 0.78 ms a frame), arrivals at 0.9 of the batch-of-8 rate: the loop
    # adds no delay to what the policy itself implies
    fixed, per = 0.07e-3, 0.78e-3
    rate = 0.9 * 8 / (fixed + 8 * per)
    fr = frames_for(1500, 1, rate=rate, seed=5, N=4, F=1, T=4)
    arrivals = [f.arrival for f in fr]
    clk = VClock()
    la = ExactLauncher(clk, arrivals, 8, slots=10_000, service_s=fixed, per_frame_s=per)
    rep = RequestLoop(la, max_inflight=max_inflight, dump_every=10_000, clock=clk,
                      sleep=clk.sleep).run(fr)
    assert rep.frames == len(fr)
    got = np.array([f.done - f.arrival for f in fr])
    want = single_server_latencies(arrivals, lambda k: fixed + per * k, max_inflight, 8)
    assert np.allclose(got, want, rtol=0, atol=1e-9)
    assert np.percentile(got, 99) > 5 * (fixed + per)  # a loaded queue, not an idle one


class RecordingMarkers:
    def __init__(self):
        self.events = []

    def push(self, message):
        self.events.append(("push", message))

    def pop(self):
        self.events.append(("pop", None))


def test_loop_opens_a_marker_range_per_run_launch_and_dump():
    clk = VClock()
    la = FakeLauncher(clk, slots=3, service_s=0.001)
    mk = RecordingMarkers()
    fr = frames_for(30, 2, rate=2000.0, seed=4)
    rep = RequestLoop(la, max_inflight=2, dump_every=6, clock=clk, sleep=clk.sleep,
                      markers=mk).run(fr)
    depth, peak = 0, 0
    for kind, _ in mk.events:  # balanced and properly nested
        depth += 1 if kind == "push" else -1
        assert depth >= 0
        peak = max(peak, depth)
    assert depth == 0 and peak == 2
    pushes = [m for kind, m in mk.events if kind == "push"]
    assert pushes[0] == "request loop: 30 frames"
    assert sum(m.startswith("launch: ") for m in pushes) == len(rep.batch_sizes)
    assert sum(m.startswith("dump: ") for m in pushes) == len(rep.dumps) > 0


def test_default_markers_load_or_do_nothing():
    from paper_1503_06202_amd.stream import Markers

    mk = Markers()  # a roctx library where ROCm is installed, else no-ops
    mk.push("test range")
    mk.pop()
