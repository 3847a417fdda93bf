#!/usr/bin/env python3
"""Benchmark of the X-engine on one MI355X.

One step = one call of the correlation over a whole frame of the full-array
workload (N = 2048 inputs, F = 16 channels, T = 32768 samples, seeded
correlated-Gaussian 4+4-bit data with 5% toned channels), inputs resident in
HBM.  Prints one JSON line: useful complex MACs per second (F T N(N+1)/2 per
frame, Eq. (1)), the fraction of the int8 MFMA peak (8 ops per complex MAC),
channels sustained in real time at the 2.56 us sample period (2^23 samples in
21.47 s), and the kernel's roofline figures, next to the CPU oracle timed on a
bounded sample of the same frame.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("complex MACs/s and % int8 MFMA peak at N=2048; channels sustained real-time; "
          "p99 frame latency")
PEAK_TOPS = {"i8": 5000.0, "f8": 5000.0}   # dense MFMA peaks of MI355X (int8 TOP/s, FP8 TFLOP/s)
HBM_GBPS = 8000.0                           # HBM3E bandwidth of MI355X, GB/s

# The sources each measured kernel is built from: a traffic figure in
# profiles/traffic.json counts only while their digest matches the one stored
# with it (counters taken on another version of the kernel are reported null).
KERNEL_SOURCES = {
    "full_array/i8": ("xcorr_device.hpp", "xcorr_plain.hip", "xcorr_tile.hpp",
                      "xeng_internal.hpp"),
    "full_array/f8": ("xcorr_device.hpp", "xcorr_plain.hip", "xcorr_tile.hpp",
                      "xeng_internal.hpp"),
    "full_array/beams16": ("xeng_beam.hip", "xeng_internal.hpp"),
    "pathfinder/i8": ("xcorr_chan.hip", "xeng_chan.hpp", "xcorr_device.hpp", "xcorr_tile.hpp",
                      "xeng_internal.hpp"),
}


def kernel_sources_sha(key):
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(key, ()):
        with open(os.path.join(ROOT, "paper_1503_06202_amd", "csrc", name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]
SAMPLE_PERIOD_S = 21.47 / 2 ** 23          # one sample per channel every 2.56 us
CHANNEL_MHZ = 400.0 / 1024                 # 1024 channels over 400 MHz


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="full_array",
                    help="full_array (default), pathfinder, precision or tiny")
    ap.add_argument("--form", default="i8", choices=["i8", "f8"])
    ap.add_argument("--split-t", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the MFMA-ceiling probe (measured MFMA throughput and clock on "
                         "Gaussian-quantised operands, reported beside the data-sheet peak)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of the frame's size (a known byte "
                         "count for scaling the HBM counters of a profiler run)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per launch (from rocprofv3 counters), if present")
    ap.add_argument("--forms",
                    default="tuner,f8,precision,pathfinder,gated,shifted,flagged,beams,batched,"
                            "stream",
                    help="other forms reported beside the headline line (comma list of tuner, "
                         "f8, precision, pathfinder, gated, shifted, flagged, beams, batched, "
                         "stream; empty for none)")
    ap.add_argument("--stream-frames", type=int, default=1000)
    return ap.parse_args()


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _time_calls(fn, steps, torch, warm_s=0.3):
    """Mean ms of `steps` calls of fn, bracketed by device synchronisation,
    after about warm_s seconds of calls: the GPU clock ramps down while the
    host generates a form's inputs, and back up under load."""
    t_warm = time.perf_counter()
    while True:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t_warm >= warm_s:
            break
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def bench_fp8(d, w, steps, torch):
    """The FP8 e4m3 form on the same frame (f32 sums flushed to int32)."""
    from paper_1503_06202_amd import Plan, vis_shape

    vis = torch.empty(vis_shape(w.N, w.F), dtype=torch.int32, device=d.device)
    with Plan(w.N, w.F, w.T, form="f8") as p:
        ms = _time_calls(lambda: p.correlate(d, vis), steps, torch)
    ops = 8.0 * w.cmac / (ms / 1e3) / 1e12
    return {"workload": w.name, "ms_per_frame": ms, "cmac_per_s": w.cmac / (ms / 1e3),
            "tflops": ops, "pct_fp8_peak": 100.0 * ops / PEAK_TOPS["f8"]}


def bench_precision(steps, torch):
    """FP8 beside int8 on the precision workload (N = 2048, F = 16,
    T = 131072; 4 GiB per frame).  The FP8 form flushes its f32 sums to int32
    every 32768 samples, i.e. four launches per frame; int8 takes the frame in
    one launch."""
    import synth
    from paper_1503_06202_amd import Plan

    w = synth.workload("precision")
    t0 = time.perf_counter()
    frame = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    _log(f"bench: precision frame generated in {time.perf_counter() - t0:.1f} s")
    out = {"workload": w.name, "N": w.N, "F": w.F, "T": w.T, "sha256": synth.frame_sha256(frame)}
    d = torch.from_numpy(frame).to("cuda:0")
    del frame
    vis = torch.empty(vis_shape_of(w), dtype=torch.int32, device=d.device)
    for form in ("f8", "i8"):
        with Plan(w.N, w.F, w.T, form=form) as p:
            ms = _time_calls(lambda: p.correlate(d, vis), max(4, steps // 2), torch)
        ops = 8.0 * w.cmac / (ms / 1e3) / 1e12
        out[form] = {"ms_per_frame": ms, "cmac_per_s": w.cmac / (ms / 1e3), "tflops": ops,
                     "pct_peak": 100.0 * ops / PEAK_TOPS[form]}
    del d, vis
    return out


def bench_gated(d, w, steps, torch, G=16, period=8192):
    """Output gating on the same frame: each sample's phase in a period of
    `period` samples picks one of G buffers (a pulsar-like fold); all G
    buffers are written once per frame."""
    import numpy as np

    from paper_1503_06202_amd import Plan

    t = np.arange(w.T, dtype=np.int64)
    gate = ((t % period) * G // period).astype(np.int32)
    vis = torch.empty((G,) + vis_shape_of(w), dtype=torch.int32, device=d.device)
    with Plan(w.N, w.F, w.T, gates=G) as p:
        ms = _time_calls(lambda: p.correlate_gated(d, gate, G, vis), steps, torch)
    out_bytes = G * 8 * w.F * w.baselines
    return {"workload": w.name, "gates": G, "period_samples": period, "ms_per_frame": ms,
            "cmac_per_s": w.cmac / (ms / 1e3), "pct_int8_peak": 100.0 * 8.0 * w.cmac / (ms / 1e3) / 1e12 / PEAK_TOPS["i8"],
            "output_bytes": out_bytes}


def bench_shifted(d, w, steps, torch, D_max=60000):
    """Time shifting on the same frame, for two delay patterns: two stations
    (inputs 0..1023 undelayed, 1024..2047 delayed 40000 samples, 102 ms) and
    the worst case, a seeded delay of 0..D_max samples for every group of 16
    inputs (D_max = 60000 is 154 ms at the 2.56 us sample period; the paper
    corrects up to 168 ms).  History rows in front of the frame repeat the
    frame's own rows."""
    import numpy as np

    from paper_1503_06202_amd import Plan

    rng = np.random.default_rng(12)
    patterns = {
        "two_stations": np.where(np.arange(w.N) < w.N // 2, 0, 40000).astype(np.int32),
        "per_16_inputs": np.repeat(rng.integers(0, D_max + 1, (w.N + 15) // 16),
                                   16)[:w.N].astype(np.int32),
    }
    # [history; frame]: the history holds frame rows again, as a ring of
    # earlier frames would (zeros there would draw less MFMA power)
    ext = torch.empty((D_max + w.T, w.F, w.N), dtype=torch.uint8, device=d.device)
    ext[D_max:].copy_(d)
    for r0 in range(0, D_max, w.T):
        n = min(w.T, D_max - r0)
        ext[D_max - r0 - n:D_max - r0].copy_(d[w.T - n:])
    frame = ext[D_max:]
    vis = torch.empty(vis_shape_of(w), dtype=torch.int32, device=d.device)
    out = {"workload": w.name, "D_max": D_max}
    with Plan(w.N, w.F, w.T) as p:
        for name, delays in patterns.items():
            p.set_delays(delays, D_max)
            ms = _time_calls(lambda: p.correlate(frame, vis), max(3, steps // 4), torch)
            out[name] = {"ms_per_frame": ms, "cmac_per_s": w.cmac / (ms / 1e3),
                         "pct_int8_peak": 100.0 * 8.0 * w.cmac / (ms / 1e3) / 1e12 / PEAK_TOPS["i8"]}
    del ext
    return out


def bench_flagged(d, w, steps, torch):
    """Flagged data on the same frame, for two seeded flag recipes: pathfinder
    (rare faults: 0.1% of packets lost, 0.1% of input blocks saturated, 1e-5 of
    samples overflowed) and heavy (5% of packets lost, 2% of input blocks
    saturated).  Reports the time of a whole flagged call (scan, correlation,
    event correlation, counts) and the rows that needed the event path."""
    import numpy as np

    import synth
    from paper_1503_06202_amd import Plan

    vis = torch.empty(vis_shape_of(w), dtype=torch.int32, device=d.device)
    counts = torch.empty((w.F, w.baselines), dtype=torch.int32, device=d.device)
    frame = d.clone()  # flagged samples are zeroed in place
    out = {"workload": w.name}
    with Plan(w.N, w.F, w.T, flagged=True) as p:
        for k, recipe in enumerate(("pathfinder", "heavy")):
            fl = synth.gen_flags(w.T, w.F, w.N, 20 + k, recipe)
            per_row = np.bitwise_count(fl).sum(axis=-1)            # invalid inputs per (t, f)
            multi = int((per_row >= 2).sum(axis=0).max())
            flags = torch.from_numpy(fl.view(np.int32)).to(d.device)
            ms = _time_calls(lambda: p.correlate_flagged(frame, flags, vis, counts),
                             max(3, steps // 4), torch)
            out[recipe] = {"ms_per_frame": ms, "invalid_fraction": float(per_row.sum()) / (w.T * w.F * w.N),
                           "event_rows_max_channel": (multi + 1) // 2,
                           "pct_int8_peak": 100.0 * 8.0 * w.cmac / (ms / 1e3) / 1e12 / PEAK_TOPS["i8"]}
            del flags
    del frame
    return out


def bench_beams(d, w, steps, torch, beam_counts=(16, 32, 64)):
    """Discrete beamforming on the same frame: B phased beams (seeded
    pointings, 127 e^{-i phi} weights) written at the sample cadence.  The path
    is bound by HBM: algorithmic bytes are the frame (T F N) plus the beams
    (8 T F B); every 64 beams read the frame once."""
    import synth
    from paper_1503_06202_amd import Plan

    out = {"workload": w.name}
    for B in beam_counts:
        y = torch.empty((w.T, w.F, B, 2), dtype=torch.int32, device=d.device)
        with Plan(w.N, w.F, w.T, beams=B) as p:
            p.set_weights(synth.gen_beam_weights(w.F, B, w.N, 7))
            ms = _time_calls(lambda: p.beamform(d, y), max(3, steps // 2), torch)
        nbytes = w.T * w.F * w.N + 8 * w.T * w.F * B
        passes = -(-2 * B // 128)   # one launch covers 64 beams
        out[f"B{B}"] = {"ms_per_frame": ms, "algorithmic_bytes": nbytes,
                        "hbm_GBps": nbytes / (ms / 1e3) / 1e9,
                        "hbm_frac": nbytes / (ms / 1e3) / 1e9 / HBM_GBPS,
                        "frame_reads": passes,
                        "int8_tops": 8.0 * B * w.N * w.T * w.F / (ms / 1e3) / 1e12}
        del y
    return out


def bench_pathfinder(steps, torch):
    """The Pathfinder shape (N = 256, F = 64, T = 32768; 512 MiB per frame):
    only about 1.6x above the int8 ridge, so both the MFMA fraction and the
    algorithmic HBM rate are reported."""
    import synth
    from paper_1503_06202_amd import Plan

    w = synth.workload("pathfinder")
    frame = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    d = torch.from_numpy(frame).to("cuda:0")
    vis = torch.empty(vis_shape_of(w), dtype=torch.int32, device=d.device)
    from paper_1503_06202_amd import tune

    with Plan(w.N, w.F, w.T) as p:
        ms = _time_calls(lambda: p.correlate(d, vis), steps, torch)
    # the tile shape and time slices the autotuner picks for this shape (on
    # this frame; every candidate's output is checked bit-identical)
    kernel, split = tune.tune_plain(w.N, w.F, w.T, cache_path=None, frame=d)
    with Plan(w.N, w.F, w.T, kernel=kernel, split_t=split) as p:
        ms_tuned = _time_calls(lambda: p.correlate(d, vis), steps, torch)
    nbytes = w.T * w.F * w.N + 8 * w.F * w.baselines
    ops = 8.0 * w.cmac / (ms / 1e3) / 1e12
    out = {"workload": w.name, "N": w.N, "F": w.F, "T": w.T, "ms_per_frame": ms,
           "cmac_per_s": w.cmac / (ms / 1e3), "pct_int8_peak": 100.0 * ops / PEAK_TOPS["i8"],
           "algorithmic_GBps": nbytes / (ms / 1e3) / 1e9,
           "hbm_frac": nbytes / (ms / 1e3) / 1e9 / HBM_GBPS,
           "realtime_channels": w.F * w.T * SAMPLE_PERIOD_S / (ms / 1e3),
           "tuned": {"kernel": kernel, "split_t": split, "ms_per_frame": ms_tuned,
                     "pct_int8_peak": 100.0 * 8.0 * w.cmac / (ms_tuned / 1e3) / 1e12 /
                     PEAK_TOPS["i8"]},
           "sha256": synth.frame_sha256(frame)}
    del d, vis
    return out


def vis_shape_of(w):
    return (w.F, w.baselines, 2)


def bench_tuner(d, w, torch):
    """The plain autotuner on the main frame: every tile shape and time-slice
    count (0 = the automatic configuration the headline step uses), timed on
    the frame, the candidates checked bit-identical to each other, and its pick."""
    from paper_1503_06202_amd import tune

    times = {}
    kernel, split = tune.tune_plain(w.N, w.F, w.T, cache_path=None, frame=d, reps=5, times=times)
    return {"workload": w.name, "kernel": kernel, "split_t": split,
            "ms_per_frame": {k: round(v, 4) for k, v in times.items()}}


def bench_batched(steps, torch):
    """48 uneven instances (N in 64..2048, T in 8192..32768, F = 4) in one graph-replayed
    persistent launch, against the plain int8 form called instance by instance."""
    import synth
    from paper_1503_06202_amd import BatchPlan, Plan, tune, vis_shape

    insts = synth.batch_instances()
    t0 = time.perf_counter()
    frames = [torch.from_numpy(synth.batch_frame(i, inst)).cuda() for i, inst in enumerate(insts)]
    _log(f"bench: batched: {len(insts)} instances generated in {time.perf_counter() - t0:.1f} s")
    vis = [torch.empty(vis_shape(N, F), dtype=torch.int32, device=frames[0].device)
           for N, F, T in insts]
    t0 = time.perf_counter()
    splits = tune.tune(insts, frames=frames, cache_path=None)
    tune_s = time.perf_counter() - t0
    cmac = sum(F * T * N * (N + 1) // 2 for N, F, T in insts)
    with BatchPlan(insts, split_t=splits) as bp:
        batched_ms = _time_calls(lambda: bp.correlate(frames, vis, graph=True), steps, torch)
        ref = [v.clone() for v in vis]
    plans = [Plan(N, F, T) for N, F, T in insts]

    def plain():
        for p, fr, v in zip(plans, frames, vis):
            p.correlate(fr, v)

    plain_ms = _time_calls(plain, steps, torch)
    same = all(torch.equal(a, b) for a, b in zip(ref, vis))
    for p in plans:
        p.close()
    return {"instances": len(insts), "cmac_per_launch": cmac, "tune_s": tune_s,
            "split_t": splits, "batched_graph_ms": batched_ms,
            "batched_cmac_per_s": cmac / (batched_ms / 1e3),
            "plain_int8_ms": plain_ms, "plain_int8_cmac_per_s": cmac / (plain_ms / 1e3),
            "batched_over_plain": plain_ms / batched_ms, "batched_equals_plain": bool(same)}


def bench_stream(n_frames, torch):
    """Request loop: frames (N=2048, F=4, T=32768) at Poisson arrivals, continuous
    batching (at most 8 frames a launch, two launches queued on one HIP
    stream, slots sized from free device memory, time slices per batch size
    tuned on the frames first), device-resident
    accumulator dumped every 256 frames into pinned buffers allocated up
    front."""
    import numpy as np

    import synth
    from paper_1503_06202_amd.stream import Frame, GpuLauncher, RequestLoop, poisson_arrivals

    w = synth.workload("stream_frame")
    pool = [torch.from_numpy(synth.stream_frame(k)).cuda() for k in range(8)]
    dump_every = 256
    launcher = GpuLauncher(w.N, w.F, w.T, streams=1, graph=True, max_batch=8, queues=1,
                           dump_buffers=n_frames // dump_every + 2)
    launcher.tune_slices(pool)
    launcher.warm(pool)
    out = {"frame": {"N": w.N, "F": w.F, "T": w.T}, "slots": launcher.slots,
           "split_t_per_batch": {str(k): v for k, v in launcher.split_t.items()},
           "split_ms_per_batch": {str(k): {str(s): round(t, 4) for s, t in v.items()}
                                  for k, v in launcher.split_ms.items()},
           "max_batch": launcher.max_batch, "hip_streams": launcher.queues, "launches_in_flight": 2,
           "distinct_frames": len(pool), "cmac_per_frame": w.cmac}

    # service time of one launch of k frames, replayed back to back on one
    # HIP stream: what a batch of k costs when it has the GPU to itself
    svc = {}
    for k in (1, 2, 4, 8):
        plan = launcher.plans[0][k]
        s = launcher.hip_streams[0]
        args = (pool[:k], [launcher.acc[0]] * k)
        for _ in range(3):
            plan.correlate(*args, stream=s, graph=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(10):
            plan.correlate(*args, stream=s, graph=True)
        e1.record(s)
        e1.synchronize()
        svc[k] = e0.elapsed_time(e1) / 10
    launcher.acc[0].zero_()
    torch.cuda.synchronize()
    out["batch_service_ms"] = {str(k): v for k, v in svc.items()}
    out["batch_frames_per_s"] = {str(k): k / (v * 1e-3) for k, v in svc.items()}

    def run(n, rate, seed):
        arr = poisson_arrivals(n, rate, seed)
        frames = [Frame(k, 0, pool[k % len(pool)], float(arr[k])) for k in range(n)]
        loop = RequestLoop(launcher, max_inflight=2, dump_every=dump_every)
        rep = loop.run(frames)
        torch.cuda.synchronize()
        return rep

    # A p99 from one sample of 1000 Poisson arrivals at rho = 0.9 depends on
    # that sample's longest busy period as much as on the loop: every load is
    # measured on several arrival samples (seeds), and the latencies of all
    # their frames are pooled.
    def run_pooled(rate, seeds):
        reps = [run(n_frames, rate, sd) for sd in seeds]
        lat = np.concatenate([r.latencies_ms for r in reps])
        batches = [b for r in reps for b in r.batch_sizes]
        return {"frames": int(lat.size), "seeds": list(seeds),
                "frames_per_s": float(lat.size / sum(r.wall_s for r in reps)),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat.max()), "mean_batch": float(np.mean(batches)),
                "launches": len(batches), "dumps": sum(len(r.dumps) for r in reps),
                "p99_ms_per_seed": [r.pct(99) for r in reps]}

    # capacity: the faster of two runs of 400 frames that all arrive at once
    # (one run alone varies by several percent from run to run)
    sats = [run(400, float("inf"), 1) for _ in range(2)]
    sat = max(sats, key=lambda r: r.frames_per_s)
    mu = sat.frames_per_s
    out["saturated"] = dict(sat.summary(), runs_frames_per_s=[r.frames_per_s for r in sats])
    out["service_rate_frames_per_s"] = mu
    out["saturated_cmac_per_s"] = mu * w.cmac
    out["poisson_rho_0.5"] = run_pooled(0.5 * mu, range(2, 6))
    out["poisson_rho_0.9"] = run_pooled(0.9 * mu, range(2, 10))
    # The same arrival samples at 0.9 of the service rate at the batch size the
    # loop forms at rho = 0.9 (interpolated between the measured batch sizes)
    # rather than at its saturated batch of 8.
    kbar = out["poisson_rho_0.9"]["mean_batch"]
    ks = sorted(svc)
    mu_k = float(np.interp(kbar, ks, [k / (svc[k] * 1e-3) for k in ks]))
    out["poisson_rho_0.9_at_batch"] = dict(run_pooled(0.9 * mu_k, range(2, 10)),
                                           service_rate_frames_per_s=mu_k, batch=kbar)
    frame_period = w.T * SAMPLE_PERIOD_S   # the sample clock: one frame every 83.9 ms
    rep = run(24, 1.0 / frame_period, 3)
    out["realtime_cadence"] = rep.summary()
    out["realtime_frame_period_ms"] = frame_period * 1e3
    launcher.close()
    return out


def mfma_ceiling():
    """The probe built beside the library (a child process): MFMA-only throughput
    and shader clock on operands like the kernels', i.e. what the matrix cores
    reach on this chip at its power limit."""
    import subprocess

    import numpy as np

    exe = os.path.join(ROOT, "paper_1503_06202_amd", "mfma_ceiling")
    if not os.path.exists(exe):
        return None
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if res.returncode != 0:
        return {"error": (res.stdout + res.stderr)[-300:]}
    return json.loads(res.stdout.strip().splitlines()[-1])


_ONE_CORE = """
import sys, time
import numpy as np
import oracle
T, N = int(sys.argv[1]), int(sys.argv[2])
s = np.frombuffer(sys.stdin.buffer.read(), np.uint8).reshape(T, 1, N)
lib = oracle.load()
t0 = time.perf_counter()
oracle.correlate(s, lib=lib)
print(time.perf_counter() - t0, oracle.threads(lib))
"""


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def one_core(frame, w, T1):
    """The oracle on one thread (OMP_NUM_THREADS=1, a child process) over the
    first T1 samples of channel 0."""
    import subprocess

    import numpy as np

    sub = np.ascontiguousarray(frame[:T1, 0, :])
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", _ONE_CORE, str(T1), str(w.N)], input=sub.tobytes(),
                         capture_output=True, env=env, cwd=os.path.dirname(os.path.abspath(__file__)),
                         timeout=300)
    if res.returncode != 0:
        return {"error": res.stderr.decode(errors="replace")[-300:]}
    dt, nthr = res.stdout.decode().split()[-2:]
    cmac = T1 * w.baselines
    return {"value": cmac / float(dt), "unit": "cMAC/s", "cores": int(nthr),
            "sample": f"channel 0, first {T1} samples ({cmac:.3e} complex MACs, {float(dt):.1f} s)"}


def cpu_baseline(frame, w, budget_s=10.0):
    """The oracle on whole channels of the same frame (all T samples each),
    channel after channel until about budget_s seconds have run, on every
    thread OpenMP takes; then on one thread over a shorter stretch of
    channel 0."""
    import oracle

    lib = oracle.load()
    dt, nch = 0.0, 0
    while nch < w.F and (nch == 0 or dt < budget_s):  # at least one whole channel
        t0 = time.perf_counter()
        oracle.correlate(frame, channels=[nch], lib=lib)
        dt += time.perf_counter() - t0
        nch += 1
    cmac = nch * w.T * w.baselines
    out = {"value": cmac / dt, "unit": "cMAC/s", "cores": oracle.threads(lib), "kind": "oracle",
           "sample": f"channels 0..{nch - 1} of the {w.name} frame ({nch} of {w.F}), all {w.T} "
                     f"samples each ({cmac:.3e} complex MACs, {dt:.1f} s)",
           "cpu": cpu_model(), "host_cpus": os.cpu_count()}
    # about 5 s on one thread at the rate just measured, in whole 256-sample steps
    per_thread = cmac / dt / max(1, out["cores"])
    T1 = int(min(w.T, max(256, 5.0 * per_thread / w.baselines // 256 * 256)))
    out["one_core"] = one_core(frame, w, T1)
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this X-engine benchmark runs on exactly one GPU.  Channels are "
              "independent, so several GPUs would each correlate their own channels with no "
              "exchange; only the one-GPU figure is measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1503_06202_amd import Plan, vis_shape

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = synth.workload(args.workload)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    frame = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    gen_s = time.perf_counter() - t0
    d = torch.from_numpy(frame).to(dev)
    vis = torch.empty(vis_shape(w.N, w.F), dtype=torch.int32, device=dev)
    plan = Plan(w.N, w.F, w.T, form=args.form, split_t=args.split_t)
    stream = torch.cuda.current_stream()
    print(f"bench: workload {w.name} N={w.N} F={w.F} T={w.T} form={args.form} "
          f"(generated in {gen_s:.1f} s)", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.correlate(d, vis, stream)
    torch.cuda.synchronize()

    # per-launch timing with events on the stream the kernels are launched on
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        plan.correlate(d, vis, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_step = wall * 1e3 / args.steps
    ev_avg = sum(ev_ms) / len(ev_ms)

    cmac = w.cmac
    value = cmac / (ms_step / 1e3)
    ops_per_launch = 8.0 * cmac          # 1 complex MAC = 4 real MACs = 8 ops
    achieved = ops_per_launch / (ev_avg / 1e3) / 1e12
    peak = PEAK_TOPS[args.form]
    frame_s = w.T * SAMPLE_PERIOD_S
    channels_rt = w.F * frame_s / (ms_step / 1e3)

    traffic = None
    traffic_note = "no counters for this kernel"
    if os.path.exists(args.traffic):
        with open(args.traffic) as fh:
            tr = json.load(fh)
        key = f"{w.name}/{args.form}"
        if key in tr:
            if tr[key].get("sources_sha256") == kernel_sources_sha(key):
                traffic = tr[key].get("bytes_per_launch")
                traffic_note = tr[key].get("source", "")
            else:
                traffic_note = "counters were taken on another version of the kernel"

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8" if args.form == "i8" else "fp8-e4m3",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "F": w.F, "T": w.T, "recipe": w.kind,
                   "seed": w.seed, "form": args.form, "baselines_per_channel": w.baselines,
                   "parallelism": "single GPU (channels independent)"},
        "pct_mfma_peak": 100.0 * achieved / peak,
        "realtime_channels": channels_rt,
        "mhz_per_gpu": channels_rt * CHANNEL_MHZ,
        "kernel_ms_avg": ev_avg,
        "kernel_ms_min": min(ev_ms),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic, "traffic_note": traffic_note},
    }
    out["config"]["sha256"] = synth.frame_sha256(frame)
    # Host-fed rate, beside (never instead of) the device-resident value: one
    # copy of the frame from pinned host memory, then the correlation.
    pinned = torch.from_numpy(frame).pin_memory()
    h2d = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        d.copy_(pinned, non_blocking=True)
        e1.record(stream)
        torch.cuda.synchronize()
        h2d.append(e0.elapsed_time(e1))
    h2d_ms = min(h2d)
    out["h2d"] = {"frame_bytes": int(d.numel()), "ms": h2d_ms,
                  "GBps": d.numel() / (h2d_ms / 1e3) / 1e9,
                  "realtime_channels_with_h2d": w.F * frame_s / ((h2d_ms + ms_step) / 1e3)}
    del pinned
    if args.calibrate_copy:
        dst = torch.empty_like(d)
        dst.copy_(d)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * d.numel()
        del dst
    plan.close()
    forms = [f for f in args.forms.split(",") if f]
    extra = {}
    if "tuner" in forms:
        _log("bench: autotuner on the main frame")
        extra["tuner"] = bench_tuner(d, w, torch)
    if "f8" in forms:
        _log("bench: fp8 form")
        extra["fp8"] = bench_fp8(d, w, args.steps, torch)
    if "precision" in forms:
        _log("bench: precision workload, fp8 and int8")
        extra["precision"] = bench_precision(args.steps, torch)
    if "pathfinder" in forms:
        _log("bench: pathfinder shape")
        extra["pathfinder"] = bench_pathfinder(args.steps, torch)
    if "gated" in forms:
        _log("bench: gated form")
        extra["gated"] = bench_gated(d, w, args.steps, torch)
    if "shifted" in forms:
        _log("bench: shifted form")
        extra["shifted"] = bench_shifted(d, w, args.steps, torch)
    if "flagged" in forms:
        _log("bench: flagged form")
        extra["flagged"] = bench_flagged(d, w, args.steps, torch)
    if "beams" in forms:
        _log("bench: beamforming form")
        extra["beams"] = bench_beams(d, w, args.steps, torch)
    if "batched" in forms:
        _log("bench: batched form")
        extra["batched"] = bench_batched(max(3, args.steps // 4), torch)
    if "stream" in forms:
        _log("bench: streaming loop")
        extra["stream"] = bench_stream(args.stream_frames, torch)
        st = extra["stream"]
        out["p99_frame_latency_ms"] = st["poisson_rho_0.9"]["p99_ms"]
        fr = st["frame"]
        out["p99_frame_latency"] = {
            "unit": "ms",
            "frames": f"N={fr['N']} F={fr['F']} T={fr['T']}, Poisson arrivals at rho times the "
                      "saturated service rate (rho_0.5, rho_0.9) or the service rate at the "
                      "loop's mean batch at rho 0.9 (rho_0.9_at_batch), latencies pooled over "
                      "several arrival samples of 1000 frames (4 at rho 0.5, 8 at rho 0.9), "
                      "or one frame per T x 2.56 us (real-time cadence)",
            "rho_0.5": st["poisson_rho_0.5"]["p99_ms"],
            "rho_0.9": st["poisson_rho_0.9"]["p99_ms"],
            "rho_0.9_at_batch": st["poisson_rho_0.9_at_batch"]["p99_ms"],
            "realtime_cadence": st["realtime_cadence"]["p99_ms"]}
    if extra:
        out["forms"] = extra
    if not args.no_ceiling:
        _log("bench: MFMA ceiling probe")
        ceil = mfma_ceiling()
        if ceil:
            out["mfma_ceiling"] = ceil
            key = "i8-codes" if args.form == "i8" else "f8-codes"
            if key in ceil and ceil[key].get("tops"):
                out["roofline"]["frac_of_measured_ceiling"] = achieved / ceil[key]["tops"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(frame, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
