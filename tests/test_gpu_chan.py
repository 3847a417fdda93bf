"""The channel kernel (one workgroup of eight waves per channel and time
slice, N <= 256, int8) against the CPU oracle, bit-exact.

Its diagonal blocks carry one accumulator D = Re + Im (plus a sum term) and
recover Re and Im from D and its transpose; its off-diagonal blocks are the
tile kernels' Re / Im pairs.  The shapes cover every quarter and fragment of
the 256-input triangle, partial fragments, ragged and single-chunk frames,
time slices, accumulation, unaligned frames (byte loads) and the integration
limits of the int32 sums.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1503_06202_amd import Plan

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def gpu(samples, split_t=0, vis=None, accumulate=False, kernel=5):
    T, F, N = samples.shape
    d = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    with Plan(N, F, T, accumulate=accumulate, split_t=split_t, kernel=kernel) as p:
        out = p.correlate(d, vis)
        torch.cuda.synchronize()
    return out.cpu().numpy()


def want(samples):
    return oracle.to_int32(oracle.correlate(samples))


def rand_frame(seed, T, F, N):
    return np.random.default_rng(seed).integers(0, 256, (T, F, N), dtype=np.uint8)


CHAN_SHAPES = [(1, 1), (17, 64), (32, 65), (64, 1000), (100, 130), (128, 128), (130, 64),
               (144, 300), (200, 257), (250, 1000), (255, 64), (256, 1), (256, 63),
               (256, 640), (256, 4133)]


@pytest.mark.parametrize("N,T", CHAN_SHAPES)
def test_chan_shapes(N, T):
    s = rand_frame(N * 977 + T, T, 3, N)
    print(f"chan N={N} F=3 T={T}", flush=True)
    assert np.array_equal(gpu(s), want(s))


@pytest.mark.parametrize("N", [144, 192, 256])
def test_chan_is_the_automatic_choice(N):
    # 128 < N <= 256, N % 16 == 0: the automatic kernel is the channel kernel
    s = rand_frame(N + 5, 2048 + 3 * 64 + 9, 4, N)
    ref = want(s)
    assert np.array_equal(gpu(s, kernel=0), ref)
    assert np.array_equal(gpu(s, kernel=0), gpu(s, kernel=1))


@pytest.mark.parametrize("split", [1, 2, 3, 7, 16])
def test_chan_time_slices(split):
    s = rand_frame(60 + split, 4133, 3, 256)
    print(f"chan slices split={split}", flush=True)
    assert np.array_equal(gpu(s, split_t=split), want(s))


@pytest.mark.parametrize("split", [1, 4])
def test_chan_accumulate(split):
    a, b = rand_frame(71, 700, 2, 240), rand_frame(72, 700, 2, 240)
    base = torch.from_numpy(want(a)).to(DEV)
    got = gpu(b, split_t=split, vis=base, accumulate=True)
    assert np.array_equal(got, want(a) + want(b))


@pytest.mark.parametrize("split,offset", [(1, 4096), (5, 4096), (5, 4097)])
def test_chan_writes_only_its_triangle(split, offset):
    # offset 4097: vis only 4-byte aligned (the slices' sum takes the
    # word-by-word path)
    T, F, N = 900, 3, 256
    s = rand_frame(73, T, F, N)
    n = F * N * (N + 1)
    sentinel = 0x5EADBEEF
    buf = torch.full((n + 2 * 4097,), sentinel, dtype=torch.int32, device=DEV)
    vis = buf[offset:offset + n].view(F, N * (N + 1) // 2, 2)
    gpu(s, split_t=split, vis=vis)
    h = buf.cpu().numpy()
    assert (h[:offset] == sentinel).all() and (h[offset + n:] == sentinel).all()
    got = vis.cpu().numpy()
    assert np.array_equal(got, want(s))
    iu, ju = np.triu_indices(N)
    assert (got[:, iu == ju, 1] == 0).all()


@pytest.mark.parametrize("split", [2, 3, 16])
def test_chan_slices_cross_zero(split):
    # time slices whose partial real parts have opposite signs, summed into vis
    # by the second kernel, also onto negative and positive starting values
    T, F, N = 64 * 48, 2, 200
    s = rand_frame(78, T, F, N)
    s[: T // 2] = 0x00            # -8-8i: large positive real parts
    s[T // 2:, :, ::2] = 0xF0     # 7-8i against -8-8i: negative real parts
    s[T // 2:, :, 1::2] = 0x00
    ref = want(s)
    assert np.array_equal(gpu(s, split_t=split), ref)
    start = np.random.default_rng(79).integers(-5_000_000, 5_000_000, ref.shape).astype(np.int32)
    vis = torch.from_numpy(start).to(DEV)
    got = gpu(s, split_t=split, vis=vis, accumulate=True)
    assert np.array_equal(got, ref + start)


def test_chan_unaligned_frame():
    # the frame starts at an odd byte: byte loads throughout
    T, F, N = 333, 2, 160
    s = rand_frame(74, T, F, N)
    raw = torch.zeros(s.size + 5, dtype=torch.uint8, device=DEV)
    view = raw[5:].view(T, F, N)
    view.copy_(torch.from_numpy(s).to(DEV))
    assert view.data_ptr() % 16 != 0
    with Plan(N, F, T, kernel=5) as p:
        got = p.correlate(view)
        torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want(s))


def test_chan_extreme_codes():
    # constant -8-8i and 7+7i: the largest visibilities, Re = 128 T and 98 T
    T, N = 65536 + 640, 256
    got = gpu(np.zeros((T, 1, N), dtype=np.uint8))
    assert (got[..., 0] == 128 * T).all() and (got[..., 1] == 0).all()
    got = gpu(np.full((T, 1, N), 0xFF, dtype=np.uint8))
    assert (got[..., 0] == 98 * T).all() and (got[..., 1] == 0).all()
    # -8-8i against 7+7i, with the sign of Im swapped on every third sample
    N = 96
    s2 = np.where(np.arange(N)[None, None, :] % 2 == 0, 0x00, 0xFF).astype(np.uint8)
    s2 = np.broadcast_to(s2, (T, 1, N)).copy()
    s2[::3] ^= 0x0F
    assert np.array_equal(gpu(s2), want(s2))


def test_chan_segment_boundary():
    # frames above 2^19 samples run as several launches (int32 sums of codes)
    T, N = (1 << 19) + 3 * 64 + 5, 72
    s = rand_frame(75, T, 1, N)
    assert np.array_equal(gpu(s), want(s))
    # the largest diagonal accumulators: codes m = r = 15 against r = 15, m = 0
    s2 = np.where(np.arange(N)[None, None, :] % 2 == 0, 0xFF, 0xF0).astype(np.uint8)
    s2 = np.broadcast_to(s2, (T, 1, N)).copy()
    assert np.array_equal(gpu(s2), want(s2))


def test_chan_rejected_outside_its_range():
    # kernel 5 on N > 256 or the FP8 form runs the 128 x 128 kernels instead
    s = rand_frame(76, 200, 2, 300)
    assert np.array_equal(gpu(s), want(s))
    d = torch.from_numpy(rand_frame(77, 200, 2, 256)).to(DEV)
    with Plan(256, 2, 200, form="f8", kernel=5) as p:
        got = p.correlate(d)
        torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want(d.cpu().numpy()))


def test_chan_workspace_grows_and_orders_streams():
    # the slices' workspace grows with the slice count (after the plan's last
    # call) and is reused when it shrinks; calls on another stream wait for
    # the previous call's sum before overwriting it
    T, F, N = 4133, 2, 256
    a, b = rand_frame(80, T, F, N), rand_frame(81, T, F, N)
    da, db = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    wa, wb = want(a), want(b)
    with Plan(N, F, T, split_t=2, kernel=5) as p:
        assert np.array_equal(p.correlate(da).cpu().numpy(), wa)
        for split in (7, 3, 16):
            p.set_tuning(split, 5)
            assert np.array_equal(p.correlate(db).cpu().numpy(), wb), split
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        v1 = torch.empty_like(torch.from_numpy(wa)).to(DEV)
        v2 = torch.empty_like(v1)
        torch.cuda.synchronize()
        for _ in range(3):
            p.correlate(da, v1, stream=s1)
            p.correlate(db, v2, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(v1.cpu().numpy(), wa)
        assert np.array_equal(v2.cpu().numpy(), wb)
