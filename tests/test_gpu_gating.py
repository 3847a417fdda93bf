"""Output gating on the GPU against the oracle's gated definition (Sec. IV-C,
"Output Gating"): every sample's gate picks the buffer its products add into.

Gates are host arrays, one int per sample; values outside 0..G-1 drop the
sample.  Expected values come from the oracle only.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1503_06202_amd import Plan

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def gated(samples, gate, G, form="i8", vis=None, accumulate=False):
    T, F, N = samples.shape
    d = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    with Plan(N, F, T, form=form, accumulate=accumulate, gates=G) as p:
        out = p.correlate_gated(d, gate, G, vis)
        torch.cuda.synchronize()
    return out.cpu().numpy()


def want(samples, gate, G):
    return oracle.to_int32(oracle.correlate_gated(samples, np.asarray(gate), G))


def periodic(T, period, G, phase=0):
    """Pulsar-like fold: the gate is the phase bin of each sample."""
    t = np.arange(T, dtype=np.int64)
    return (((t + phase) % period) * G // period).astype(np.int32)


def rand_frame(seed, T, F, N):
    return np.random.default_rng(seed).integers(0, 256, (T, F, N), dtype=np.uint8)


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_random_gates_short_runs(form):
    T, F, N, G = 700, 2, 72, 3
    s = rand_frame(51, T, F, N)
    gate = np.random.default_rng(52).integers(-1, G + 1, T).astype(np.int32)  # -1 and G drop
    assert np.array_equal(gated(s, gate, G, form), want(s, gate, G))


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_periodic_fold(form):
    T, F, N, G = 32768 + 37, 4, 256, 8
    s = synth.gen_frame(N, F, T, 2, "gauss")
    gate = periodic(T, 3001, G, phase=123)
    assert np.array_equal(gated(s, gate, G, form), want(s, gate, G))


def test_accumulate_and_empty_gates():
    T, F, N, G = 1000, 1, 40, 5
    s = rand_frame(53, T, F, N)
    gate = np.where(np.arange(T) < 500, 1, 3).astype(np.int32)  # gates 0, 2, 4 stay empty
    ref = want(s, gate, G)
    assert not ref[0].any() and not ref[2].any()
    vis = torch.from_numpy(np.full(ref.shape, 5, dtype=np.int32)).to(DEV)
    assert np.array_equal(gated(s, gate, G, vis=vis, accumulate=True), ref + 5)
    assert np.array_equal(gated(s, gate, G), ref)


@pytest.mark.parametrize("form,T,N", [("f8", 2 * 32768 + 100, 40), ("i8", (1 << 19) + 1000, 24)])
def test_gates_across_launch_segments(form, T, N):
    # frames longer than one launch may integrate are cut into launches that
    # add; runs that straddle a cut are split there
    s = rand_frame(54, T, 1, N)
    gate = periodic(T, 20011, 4, phase=7)
    assert np.array_equal(gated(s, gate, 4, form), want(s, gate, 4))


@pytest.mark.parametrize("form,T", [("f8", 32768 + 100), ("i8", (1 << 19) + 1000)])
def test_per_sample_gates_long_frame(form, T):
    # runs of one or two samples, each integrated as a whole chunk of 64: a
    # gate holds far more chunk-rounded samples per launch segment than one
    # exact integration may (32768 in FP8, 2^19 in int8), so it is split
    # into work gates that add atomically; gate 2 has long runs only and is
    # not split
    N, F, G = 64, 2, 3
    s = rand_frame(56, T, F, N)
    gate = np.random.default_rng(57).integers(-1, 2, T).astype(np.int32)  # -1 drops
    gate[(np.arange(T) // 1000) % 5 == 4] = 2
    ref = want(s, gate, G)
    print(f"per-sample gates form={form} T={T}", flush=True)
    assert np.array_equal(gated(s, gate, G, form), ref)
    vis = torch.from_numpy(np.full(ref.shape, -3, dtype=np.int32)).to(DEV)
    assert np.array_equal(gated(s, gate, G, form, vis=vis, accumulate=True), ref - 3)


def test_gates_sum_to_ungated():
    T, F, N, G = 4096 + 64, 8, 512, 6
    s = synth.gen_frame(N, F, T, 9, "gauss")
    gate = periodic(T, 1000, G)
    g = gated(s, gate, G)
    d = torch.from_numpy(s).to(DEV)
    with Plan(N, F, T) as p:
        ungated = p.correlate(d).cpu().numpy()
    assert np.array_equal(g.astype(np.int64).sum(axis=0), ungated.astype(np.int64))


def test_full_array_sixteen_phase_bins_sampled():
    w = synth.workload("full_array")
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    G = 16
    gate = periodic(w.T, 8192, G, phase=1000)
    got = gated(s, gate, G)
    rng = np.random.default_rng(55)
    f = rng.integers(0, w.F, 40)
    i = rng.integers(0, w.N, 40)
    j = rng.integers(0, w.N, 40)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    b = lo * w.N - lo * (lo - 1) // 2 + (hi - lo)
    for g in (0, 5, 15):
        ref = oracle.correlate_pairs(s[gate == g], f, lo, hi)
        assert np.array_equal(got[g][f, b].astype(np.int64), ref), g
