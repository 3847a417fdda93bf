"""Discrete beamforming on the GPU against the oracle's definition (Sec. IV-C,
"Discrete Beamforming"): y[t][f][b] = sum_n w[f][b][n] x[t][f][n], exact.

Expected values come from ``oracle.beamform`` on the same seeded bytes and
weights (on sampled times for the full-size frames).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1503_06202_amd import Plan, _lib

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def rand_frame(seed, T, F, N):
    return np.random.default_rng(seed).integers(0, 256, (T, F, N), dtype=np.uint8)


def rand_weights(seed, F, B, N):
    return np.random.default_rng(seed).integers(-127, 128, (F, B, N, 2)).astype(np.int8)


def gpu_beams(s, w, plan=None, view=None):
    T, F, N = s.shape
    B = w.shape[1]
    d = torch.from_numpy(np.ascontiguousarray(s)).to(DEV) if view is None else view
    own = plan is None
    p = plan or Plan(N, F, T, beams=B)
    try:
        p.set_weights(w)
        y = p.beamform(d)
        torch.cuda.synchronize()
        return y.cpu().numpy()
    finally:
        if own:
            p.close()


def want(s, w):
    return oracle.beamform(s, w).astype(np.int32)


@pytest.mark.parametrize("N,T,B", [(96, 300, 5), (40, 129, 3), (64, 512, 16), (128, 77, 17),
                                   (256, 1000, 40), (2048, 200, 64), (17, 33, 1),
                                   (128, 301, 64), (512, 259, 50), (256, 300, 100),
                                   (48, 200, 57)])
def test_beams_match_oracle(N, T, B):
    F = 3
    s = rand_frame(200 + N + B, T, F, N)
    w = rand_weights(201 + N + B, F, B, N)
    print(f"beams N={N} T={T} F={F} B={B}", flush=True)
    assert np.array_equal(gpu_beams(s, w), want(s, w))


def test_extreme_codes_and_weights():
    """All samples -8-8i and weights +-127: the largest magnitudes of a beam."""
    T, F, N, B = 70, 2, 512, 4
    s = np.zeros((T, F, N), np.uint8)          # code 0: value -8 - 8i
    s[1::2] = 0xFF                             # 7 + 7i
    w = np.full((F, B, N, 2), 127, np.int8)
    w[:, 1, :, 1] = -127
    w[:, 2] = -127
    assert np.array_equal(gpu_beams(s, w), want(s, w))


def test_selection_beam_is_the_input():
    T, F, N, B = 300, 2, 160, 6
    s = rand_frame(202, T, F, N)
    w = np.zeros((F, B, N, 2), np.int8)
    for b in range(B):
        w[:, b, 7 * b + 3, 0] = 1
    y = gpu_beams(s, w)
    for b in range(B):
        n = 7 * b + 3
        assert np.array_equal(y[:, :, b, 0], (s[:, :, n] >> 4).astype(np.int32) - 8)
        assert np.array_equal(y[:, :, b, 1], (s[:, :, n] & 15).astype(np.int32) - 8)


def test_unaligned_samples_pointer():
    T, F, N, B = 260, 2, 64, 8
    s = rand_frame(203, T, F, N)
    w = rand_weights(204, F, B, N)
    buf = torch.zeros(s.size + 1, dtype=torch.uint8, device=DEV)
    buf[1:] = torch.from_numpy(s.reshape(-1)).to(DEV)
    view = buf[1:].view(T, F, N)
    assert view.data_ptr() % 16 == 1
    assert np.array_equal(gpu_beams(s, w, view=view), want(s, w))


def test_reweighting_a_plan():
    T, F, N, B = 400, 2, 128, 12
    s = rand_frame(205, T, F, N)
    with Plan(N, F, T, beams=B) as p:
        for seed in (206, 207):
            w = rand_weights(seed, F, B, N)
            assert np.array_equal(gpu_beams(s, w, plan=p), want(s, w)), seed


def test_errors():
    T, F, N, B = 64, 1, 32, 2
    s = torch.zeros((T, F, N), dtype=torch.uint8, device=DEV)
    with Plan(N, F, T, beams=B) as p:
        with pytest.raises(_lib.XengError):
            p.beamform(s)                                   # no weights yet
        w = np.zeros((F, B, N, 2), np.int8)
        w[0, 0, 0, 0] = -128
        with pytest.raises(_lib.XengError):
            p.set_weights(w)


def test_launch_segments():
    """F N = 2^21: one launch covers fewer rows than the frame, which is then
    beamformed in three launches; times near every boundary are checked."""
    F, N, B = 64, 32768, 4
    seg = ((1 << 31) - 1 - 256) // (F * N) - 512 - 2
    T = 2 * seg + 100
    rng = np.random.default_rng(208)
    block = rng.integers(0, 256, (97, F, N), dtype=np.uint8)
    s = np.ascontiguousarray(np.tile(block, (T // 97 + 1, 1, 1))[:T])
    s[::5] ^= 0x5A                                         # break the period
    w = rand_weights(209, F, B, N)
    print(f"beam segments T={T} seg={seg}", flush=True)
    y = gpu_beams(s, w)
    ts = np.array(sorted({0, 1, seg - 1, seg, seg + 1, 2 * seg - 1, 2 * seg, T - 1, 123, 700}))
    assert np.array_equal(y[ts], want(s[ts], w))


def test_full_array_sampled_times():
    """The full-array frame (N=2048, F=16, T=32768) with 16 phased beams:
    200 sampled times (all channels and beams) against the oracle."""
    w_ = synth.workload("full_array")
    s = synth.gen_frame(w_.N, w_.F, w_.T, w_.seed, w_.kind)
    wts = synth.gen_beam_weights(w_.F, 16, w_.N, 7)
    print(f"full_array beams N={w_.N} F={w_.F} T={w_.T} B=16", flush=True)
    y = gpu_beams(s, wts)
    rng = np.random.default_rng(210)
    ts = np.unique(np.concatenate([rng.integers(0, w_.T, 196), [0, 1, w_.T - 2, w_.T - 1]]))
    assert np.array_equal(y[ts], want(s[ts], wts))
