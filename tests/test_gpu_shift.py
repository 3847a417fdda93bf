"""Time shifting on the GPU against the oracle's shifted definition (Sec.
IV-C, "Time Shifting"): input n is read D delays[n] samples late; rows
before the frame come from the history kept in memory right before it.

Two paths: delays equal within every 128-input block are applied in the
kernels' loads (`block_delays`); delays that differ inside a block go through
a shifted copy of the frame (`group_delays`).  Both are tested.

A device buffer holds [history; frame]; the plan correlates the view that
starts D_max rows in.  Expected values come from the oracle only.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1503_06202_amd import Plan

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def group_delays(seed, N, D_max, zero_some=True):
    """One delay per aligned group of 16 inputs."""
    rng = np.random.default_rng(seed)
    g = rng.integers(0, D_max + 1, (N + 15) // 16)
    if zero_some:
        g[::3] = 0
    return np.repeat(g, 16)[:N].astype(np.int32)


def block_delays(seed, N, D_max):
    """One delay per aligned block of 128 inputs (the in-load path)."""
    rng = np.random.default_rng(seed)
    g = rng.integers(0, D_max + 1, (N + 127) // 128)
    g[0] = 0
    return np.repeat(g, 128)[:N].astype(np.int32)


def shifted(ext, D, delays, form="i8", vis=None, accumulate=False, gate=None, G=0):
    TT, F, N = ext.shape
    T = TT - D
    dev = torch.from_numpy(np.ascontiguousarray(ext)).to(DEV)
    frame = dev[D:]  # contiguous view: D_max rows of history in front of it
    with Plan(N, F, T, form=form, accumulate=accumulate, gates=G) as p:
        p.set_delays(delays, D)
        out = p.correlate_gated(frame, gate, G, vis) if G else p.correlate(frame, vis)
        torch.cuda.synchronize()
    return out.cpu().numpy()


def want(ext, D, delays):
    return oracle.to_int32(oracle.correlate_shifted(ext, D, delays))


def rand_ext(seed, TT, F, N):
    return np.random.default_rng(seed).integers(0, 256, (TT, F, N), dtype=np.uint8)


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("N", [96, 40, 144, 300])
def test_group_delays(form, N):
    D, T, F = 300, 700 + 5, 2
    ext = rand_ext(61 + N, D + T, F, N)
    d = group_delays(62, N, D)
    assert np.array_equal(shifted(ext, D, d, form), want(ext, D, d))


def test_zero_delays_equal_plain():
    D, T, F, N = 64, 1000, 2, 64
    ext = rand_ext(63, D + T, F, N)
    d = np.zeros(N, np.int32)
    got = shifted(ext, D, d)
    assert np.array_equal(got, oracle.to_int32(oracle.correlate(ext[D:])))


def test_pathfinder_shape_with_delays():
    w = synth.workload("pathfinder")
    D = 1000
    ext = synth.gen_frame(w.N, w.F, D + w.T, w.seed, w.kind)
    d = group_delays(64, w.N, D)
    assert np.array_equal(shifted(ext, D, d), want(ext, D, d))


def test_accumulate_and_gated_with_delays():
    D, T, F, N, G = 200, 3000, 1, 48, 3
    ext = rand_ext(65, D + T, F, N)
    d = group_delays(66, N, D, zero_some=False)
    ref = want(ext, D, d)
    vis = torch.from_numpy(np.full(ref.shape, -3, dtype=np.int32)).to(DEV)
    assert np.array_equal(shifted(ext, D, d, vis=vis, accumulate=True), ref - 3)
    gate = (np.arange(T) // 250 % G).astype(np.int32)
    got = shifted(ext, D, d, gate=gate, G=G)
    # each gate: the oracle's gated sums of the explicitly shifted samples
    xs = ext[D + np.arange(T)[:, None] - d[None, :], :, np.arange(N)[None, :]]  # [T][N][F]
    xs = np.ascontiguousarray(np.transpose(xs, (0, 2, 1)))                      # [T][F][N]
    assert np.array_equal(got, oracle.to_int32(oracle.correlate_gated(xs, gate, G)))
    assert np.array_equal(got.astype(np.int64).sum(axis=0), oracle.correlate_shifted(ext, D, d))


def test_delays_off_again():
    D, T, F, N = 32, 500, 1, 32
    ext = rand_ext(67, D + T, F, N)
    dev = torch.from_numpy(ext).to(DEV)
    with Plan(N, F, T) as p:
        p.set_delays(group_delays(68, N, D, zero_some=False), D)
        p.set_delays(None)
        got = p.correlate(dev[D:]).cpu().numpy()
    assert np.array_equal(got, oracle.to_int32(oracle.correlate(ext[D:])))


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("N", [256, 200])
def test_block_delays_in_loads(form, N):
    """Delays constant over each 128-input block: applied in the loads."""
    D, T, F = 500, 1300, 2
    ext = rand_ext(69 + N, D + T, F, N)
    d = block_delays(70, N, D)
    assert len(set(d.tolist())) > 1
    assert np.array_equal(shifted(ext, D, d, form), want(ext, D, d))


def test_switch_between_paths():
    """One plan: fine delays (copy), block delays (loads), fine again."""
    D, T, F, N = 100, 700, 2, 256
    ext = rand_ext(71, D + T, F, N)
    dev = torch.from_numpy(ext).to(DEV)
    with Plan(N, F, T) as p:
        for d in (group_delays(72, N, D), block_delays(73, N, D), group_delays(74, N, D)):
            p.set_delays(d, D)
            got = p.correlate(dev[D:]).cpu().numpy()
            assert np.array_equal(got, want(ext, D, d))


def test_gated_block_delays():
    D, T, F, N, G = 300, 2000, 1, 256, 2
    ext = rand_ext(75, D + T, F, N)
    d = block_delays(76, N, D)
    gate = (np.arange(T) // 300 % G).astype(np.int32)
    got = shifted(ext, D, d, gate=gate, G=G)
    xs = ext[D + np.arange(T)[:, None] - d[None, :], :, np.arange(N)[None, :]]
    xs = np.ascontiguousarray(np.transpose(xs, (0, 2, 1)))
    assert np.array_equal(got, oracle.to_int32(oracle.correlate_gated(xs, gate, G)))
