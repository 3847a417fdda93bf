"""Parity of the HIP X-engine with the CPU oracle (bit-exact: integer work).

Every GPU call goes through the C ABI (libxeng.so) via the package's ctypes
binding.  Inputs come from the seeded generator; expected values from the
oracle only.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1503_06202_amd import BatchPlan, Plan, engine

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def gpu(samples: np.ndarray, form="i8", split_t=0, vis=None, accumulate=False, kernel=0):
    T, F, N = samples.shape
    d = torch.from_numpy(np.ascontiguousarray(samples)).to(DEV)
    with Plan(N, F, T, form=form, accumulate=accumulate, split_t=split_t, kernel=kernel) as p:
        out = p.correlate(d, vis)
        torch.cuda.synchronize()
    return out.cpu().numpy()


def want(samples, **kw):
    return oracle.to_int32(oracle.correlate(samples, **kw))


def rand_frame(seed, T, F, N):
    return np.random.default_rng(seed).integers(0, 256, (T, F, N), dtype=np.uint8)


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_tiny_workload(form):
    w = synth.workload("tiny")
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    print(f"tiny N={w.N} F={w.F} T={w.T} form={form}", flush=True)
    assert np.array_equal(gpu(s, form), want(s))


SHAPES = [(1, 1), (2, 3), (8, 64), (15, 65), (17, 257), (33, 63), (64, 1), (127, 300),
          (128, 128), (129, 97), (200, 513), (255, 64), (256, 1000), (257, 129), (384, 200),
          (520, 130)]


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("N,T", SHAPES)
def test_odd_shapes(N, T, form):
    s = rand_frame(N * 1000 + T, T, 2, N)
    print(f"odd N={N} F=2 T={T} form={form}", flush=True)
    assert np.array_equal(gpu(s, form), want(s))


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("N,T", [(1040, 200), (1152, 130), (1090, 64)])
def test_large_n_diagonal_roles(N, T, form):
    # above 1024 inputs the diagonal tiles of 16-aligned frames keep the
    # off-diagonal wave roles (the wave below the diagonal only sums); below,
    # and for unaligned frames, two waves share the sub-tile above the diagonal
    s = rand_frame(N + T, T, 1, N)
    print(f"large N={N} T={T} form={form}", flush=True)
    assert np.array_equal(gpu(s, form), want(s))


WIDE_SHAPES = [(16, 64), (48, 65), (144, 300), (256, 129), (272, 1000), (400, 64), (512, 257),
               (640, 130)]


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("N,T", WIDE_SHAPES)
def test_wide_tiles(N, T, form):
    # the 128 x 256 tile kernel forced on shapes that cover every tile row kind
    s = rand_frame(N * 7 + T, T, 2, N)
    print(f"wide N={N} F=2 T={T} form={form}", flush=True)
    assert np.array_equal(gpu(s, form, kernel=2), want(s))


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("split", [1, 3])
def test_wide_vs_narrow_slices(split, form):
    s = synth.gen_frame(768, 2, 1500, 12, "gauss+tone")
    ref = want(s)
    assert np.array_equal(gpu(s, form, split_t=split, kernel=2), ref)
    assert np.array_equal(gpu(s, form, split_t=split, kernel=1), ref)


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("split", [1, 2, 3, 7, 32])
def test_time_slices(split, form):
    s = synth.gen_frame(257, 3, 2000, 7, "gauss+tone")
    print(f"slices split={split} form={form}", flush=True)
    assert np.array_equal(gpu(s, form, split_t=split), want(s))


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_unaligned_samples_pointer(form):
    # N % 8 == 0 but the frame starts at an odd byte: the byte-load path runs
    T, F, N = 150, 2, 64
    s = rand_frame(5, T, F, N)
    raw = torch.zeros(s.size + 3, dtype=torch.uint8, device=DEV)
    view = raw[3:].view(T, F, N)
    view.copy_(torch.from_numpy(s).to(DEV))
    assert view.data_ptr() % 8 != 0
    with Plan(N, F, T, form=form) as p:
        got = p.correlate(view)
        torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want(s))


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("split", [1, 4])
def test_accumulate_adds(form, split):
    a = rand_frame(11, 300, 2, 140)
    b = rand_frame(12, 300, 2, 140)
    base = torch.from_numpy(want(a)).to(DEV)
    got = gpu(b, form, split_t=split, vis=base, accumulate=True)
    assert np.array_equal(got, want(a) + want(b))


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("split", [1, 5])
def test_canary_guards_and_diagonal(form, split):
    T, F, N = 200, 3, 150
    s = rand_frame(13, T, F, N)
    n = F * N * (N + 1)
    sentinel = 0x5EADBEEF
    buf = torch.full((n + 2 * 4096,), sentinel, dtype=torch.int32, device=DEV)
    vis = buf[4096:4096 + n].view(F, N * (N + 1) // 2, 2)
    d = torch.from_numpy(s).to(DEV)
    with Plan(N, F, T, form=form, split_t=split) as p:
        p.correlate(d, vis)
        torch.cuda.synchronize()
    h = buf.cpu().numpy()
    assert (h[:4096] == sentinel).all() and (h[-4096:] == sentinel).all()
    got = vis.cpu().numpy()
    assert np.array_equal(got, want(s))
    iu, ju = np.triu_indices(N)
    assert (got[:, iu == ju, 1] == 0).all()


def test_repeatable_across_runs_and_forms():
    s = synth.gen_frame(300, 4, 3000, 21, "gauss+tone")
    runs = [gpu(s, "i8") for _ in range(3)] + [gpu(s, "i8", split_t=6), gpu(s, "f8"),
                                               gpu(s, "f8", split_t=3)]
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
    assert np.array_equal(runs[0], want(s))


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_extreme_codes_long_integration(form):
    # all -8-8i: the largest visibilities (128 T), carried by the offset terms
    T, N = 65536 + 640, 40
    s = np.zeros((T, 1, N), dtype=np.uint8)
    got = gpu(s, form)
    assert (got[..., 0] == 128 * T).all() and (got[..., 1] == 0).all()
    # all 7+7i: the largest sums of codes (2 * 15 * 15 per sample)
    got = gpu(np.full((T, 1, N), 0xFF, dtype=np.uint8), form)
    assert (got[..., 0] == 98 * T).all() and (got[..., 1] == 0).all()
    # mixed extremes: -8-8i against 7+7i, the largest |Im| terms
    s2 = np.where(np.arange(N)[None, None, :] % 2 == 0, 0x00, 0xFF).astype(np.uint8)
    s2 = np.broadcast_to(s2, (T, 1, N)).copy()
    s2[::3] ^= 0x0F  # swap the sign of Im on every third sample
    assert np.array_equal(gpu(s2, form), want(s2))


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_fp8_segment_boundary_random(form):
    T, F, N = 65536 + 3 * 64 + 5, 1, 72
    s = rand_frame(31, T, F, N)
    assert np.array_equal(gpu(s, form), want(s))


@pytest.mark.parametrize("form", ["i8", "f8"])
def test_head_tail_split(form):
    # 640 tiles on 512 resident workgroups: one round of whole tiles, then the
    # remaining 128 tiles in time slices that add atomically into a cleared
    # region (the automatic schedule when tiles do not divide into rounds)
    T, F, N = 4096 + 3 * 64 + 5, 64, 512
    s = rand_frame(41, T, F, N)
    ref = want(s)
    assert np.array_equal(gpu(s, form), ref)
    # accumulating: whole tiles add, tail slices add atomically
    vis = torch.from_numpy(np.full(ref.shape, 7, dtype=np.int32)).to(DEV)
    got = gpu(s, form, vis=vis, accumulate=True)
    assert np.array_equal(got, ref + 7)


def test_int8_segment_boundary():
    # the int8 128 x 128 kernels hold 16 V in int32 and split a frame into
    # launches (and a batch instance into slices) of at most 2^19 samples
    T, N = (1 << 19) + 3 * 64 + 5, 72
    s = rand_frame(37, T, 1, N)
    ref = want(s)
    assert np.array_equal(gpu(s), ref)
    d = torch.from_numpy(s).to(DEV)
    vis = torch.empty(engine.vis_shape(N, 1), dtype=torch.int32, device=DEV)
    with BatchPlan([(N, 1, T)], split_t=[1]) as bp:
        bp.correlate([d], [vis])
        torch.cuda.synchronize()
    assert np.array_equal(vis.cpu().numpy(), ref)
    # extremes on both sides of the boundary: -8-8i against 7+7i
    s2 = np.where(np.arange(N)[None, None, :] % 2 == 0, 0x00, 0xFF).astype(np.uint8)
    s2 = np.broadcast_to(s2, (T, 1, N)).copy()
    s2[::3] ^= 0x0F
    assert np.array_equal(gpu(s2), want(s2))


def test_int32_boundary():
    # T = 2^24 - 1 of -8-8i: Re = 2,147,483,520, the largest exact integration
    T, N = (1 << 24) - 1, 8
    d = torch.zeros((T, 1, N), dtype=torch.uint8, device=DEV)
    with Plan(N, 1, T) as p:
        got = p.correlate(d)
        torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert (got[..., 0] == 2147483520).all() and (got[..., 1] == 0).all()
    with Plan(N, 1, T) as p:
        with pytest.raises(engine.XengError):
            p.correlate(torch.zeros((T + 1, 1, N), dtype=torch.uint8, device=DEV))


def _sample_baselines(N, F, count, seed):
    rng = np.random.default_rng(seed)
    edges = sorted({0, 1, 31, 32, 63, 64, 127, 128, 129, N // 2, N - 2, N - 1} & set(range(N)))
    pairs = [(i, j) for i in edges for j in edges if i <= j]
    i = rng.integers(0, N, count)
    j = rng.integers(0, N, count)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    pairs += list(zip(lo.tolist(), hi.tolist()))
    f = np.concatenate([np.arange(len(pairs)) % F])
    pi = np.array([p[0] for p in pairs])
    pj = np.array([p[1] for p in pairs])
    return f, pi, pj


@pytest.fixture(scope="module")
def full_array_frame():
    w = synth.workload("full_array")
    return w, synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)


@pytest.fixture(scope="module")
def pathfinder_frame():
    w = synth.workload("pathfinder")
    return w, synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)


def _check_sampled(s, got, count, seed):
    T, F, N = s.shape
    f, i, j = _sample_baselines(N, F, count, seed)
    ref = oracle.correlate_pairs(s, f, i, j)
    b = i * N - i * (i - 1) // 2 + (j - i)
    assert np.array_equal(got[f, b].astype(np.int64), ref)
    # autocorrelations: real, equal to sum |x|^2, computed from the bytes here
    re = (s >> 4).astype(np.int64) - 8
    im = (s & 15).astype(np.int64) - 8
    power = (re * re + im * im).sum(axis=0)  # [F][N]
    d = np.arange(N) * N - np.arange(N) * (np.arange(N) - 1) // 2
    assert np.array_equal(got[:, d, 0].astype(np.int64), power)
    assert (got[:, d, 1] == 0).all()


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("kernel", [0, 1])
def test_full_array_workload_sampled(full_array_frame, form, kernel):
    w, s = full_array_frame
    print(f"full_array N={w.N} F={w.F} T={w.T} form={form} kernel={kernel}", flush=True)
    got = gpu(s, form, kernel=kernel)
    _check_sampled(s, got, 3000, 1)


def test_full_array_time_additivity(full_array_frame):
    w, s = full_array_frame
    d = torch.from_numpy(s).to(DEV)
    cut = 12345
    with Plan(w.N, w.F, w.T) as p:
        whole = p.correlate(d).cpu().numpy()
        a = p.correlate(d[:cut].contiguous()).cpu().numpy()
        b = p.correlate(d[cut:].contiguous()).cpu().numpy()
    assert np.array_equal(a.astype(np.int64) + b, whole)


def test_pathfinder_workload(pathfinder_frame):
    w, s = pathfinder_frame
    print(f"pathfinder N={w.N} F={w.F} T={w.T}", flush=True)
    got = gpu(s, "i8")
    ch = [0, 17, 63]
    assert np.array_equal(got[ch], want(s, channels=ch))
    _check_sampled(s, got, 2000, 2)
    assert np.array_equal(gpu(s, "f8"), got)


def test_precision_workload_two_channels():
    # the FP8 workload's shape (N=2048, T=131072) on a two-channel subset
    w = synth.workload("precision")
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind, channels=[0, 1])
    g8 = gpu(s, "i8")
    gf = gpu(s, "f8")
    assert np.array_equal(g8, gf)
    _check_sampled(s, gf, 1500, 3)


# ------------------------------------------------------------------ batched form
BATCH = [(1, 1, 64), (17, 2, 100), (64, 4, 1000), (130, 1, 257), (256, 2, 640), (9, 3, 7),
         (300, 1, 2000), (64, 1, 64)]


def _batch_inputs(seed=0):
    frames = [rand_frame(seed * 100 + k, T, F, N) for k, (N, F, T) in enumerate(BATCH)]
    d = [torch.from_numpy(x).to(DEV) for x in frames]
    return frames, d


def _new_vis():
    return [torch.empty(engine.vis_shape(N, F), dtype=torch.int32, device=DEV) for N, F, T in BATCH]


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("splits", [None, [1, 2, 3, 1, 4, 1, 2, 5]])
def test_batch_matches_oracle(form, splits):
    frames, d = _batch_inputs()
    vis = _new_vis()
    with BatchPlan(BATCH, form=form, split_t=splits) as bp:
        bp.correlate(d, vis)
        torch.cuda.synchronize()
    for k, s in enumerate(frames):
        assert np.array_equal(vis[k].cpu().numpy(), want(s)), k


def test_batch_alone_equals_in_mix():
    frames, d = _batch_inputs(1)
    vis = _new_vis()
    with BatchPlan(BATCH) as bp:
        bp.correlate(d, vis)
    for k, (N, F, T) in enumerate(BATCH):
        with Plan(N, F, T) as p:
            alone = p.correlate(d[k])
        assert torch.equal(alone, vis[k]), k


def test_batch_graph_replays():
    frames, d = _batch_inputs(2)
    ref = [torch.from_numpy(want(s)).to(DEV) for s in frames]
    with BatchPlan(BATCH, split_t=[1, 2, 3, 1, 4, 1, 2, 5]) as bp:
        vis = _new_vis()
        for rep in range(4):
            for v in vis:
                v.fill_(-1)
            bp.correlate(d, vis, graph=True)
            torch.cuda.synchronize()
            for k in range(len(BATCH)):
                assert torch.equal(vis[k], ref[k]), (rep, k)
            # eager work between replays
            _ = torch.ones(1000, device=DEV).sum().item()
        # new buffers: the pointer table is refreshed, the graph reused
        vis2 = _new_vis()
        bp.correlate(d, vis2, graph=True)
        torch.cuda.synchronize()
        for k in range(len(BATCH)):
            assert torch.equal(vis2[k], ref[k]), k


def test_batch_accumulate_time_additivity():
    frames, d = _batch_inputs(3)
    halves = [(x[: x.shape[0] // 2], x[x.shape[0] // 2:]) for x in d]
    inst_a = [(N, F, h[0].shape[0]) for (N, F, T), h in zip(BATCH, halves)]
    inst_b = [(N, F, h[1].shape[0]) for (N, F, T), h in zip(BATCH, halves)]
    keep = [k for k, (a, b) in enumerate(zip(inst_a, inst_b)) if a[2] > 0 and b[2] > 0]
    vis = [torch.zeros(engine.vis_shape(BATCH[k][0], BATCH[k][1]), dtype=torch.int32, device=DEV)
           for k in keep]
    with BatchPlan([inst_a[k] for k in keep], accumulate=True) as pa, \
            BatchPlan([inst_b[k] for k in keep], accumulate=True) as pb:
        pa.correlate([halves[k][0].contiguous() for k in keep], vis)
        pb.correlate([halves[k][1].contiguous() for k in keep], vis)
        torch.cuda.synchronize()
    for v, k in zip(vis, keep):
        assert np.array_equal(v.cpu().numpy(), want(frames[k])), k


@pytest.mark.parametrize("offset", [4096, 4097])
def test_batch_slices_cross_zero_and_alignment(offset):
    # time-sliced instances whose partial real parts change sign from slice to
    # slice, accumulated onto starting values of both signs: with vis 8-byte
    # aligned (offset 4096) the slices add with 64-bit atomics, whose borrows
    # between the words the fix-ups undo; at offset 4097 (4-byte aligned) with
    # 32-bit atomics.  Nothing outside the outputs is written.
    insts = [(200, 2, 64 * 48), (72, 3, 64 * 30 + 7)]
    frames = []
    for k, (N, F, T) in enumerate(insts):
        s = rand_frame(90 + k, T, F, N)
        s[: T // 2] = 0x00            # -8-8i: large positive real parts
        s[T // 2:, :, ::2] = 0xF0     # 7-8i against -8-8i: negative real parts
        s[T // 2:, :, 1::2] = 0x00
        frames.append(s)
    sizes = [F * N * (N + 1) for N, F, T in insts]
    sentinel = 0x5EADBEEF
    bufs, vis, starts = [], [], []
    rng = np.random.default_rng(91)
    for (N, F, T), n in zip(insts, sizes):
        buf = torch.full((n + 2 * 4097,), sentinel, dtype=torch.int32, device=DEV)
        start = rng.integers(-5_000_000, 5_000_000, n).astype(np.int32)
        v = buf[offset:offset + n]
        v.copy_(torch.from_numpy(start).to(DEV))
        bufs.append(buf)
        starts.append(start.reshape(engine.vis_shape(N, F)))
        vis.append(v.view(engine.vis_shape(N, F)))
    d = [torch.from_numpy(s).to(DEV) for s in frames]
    with BatchPlan(insts, accumulate=True, split_t=[3, 5]) as bp:
        bp.correlate(d, vis)
        torch.cuda.synchronize()
    for k, s in enumerate(frames):
        assert np.array_equal(vis[k].cpu().numpy(), want(s) + starts[k]), k
        h = bufs[k].cpu().numpy()
        assert (h[:offset] == sentinel).all() and (h[offset + sizes[k]:] == sentinel).all()


# Batches that leave their time slices to the library and hold a few more tiles
# than the GPU has workgroup slots: on a 256-CU GPU (512 slots) the 672 tiles
# of BIG_MIX take 3 automatic slices and the 576 of BIG_SAME 4 (cost model of
# the automatic slice count), so every tile adds its slices with atomics into a
# cleared output, or into the caller's accumulator.
BIG_MIX = [(1024, 12, 8192), (640, 16, 8192)]
BIG_SAME = [(1024, 8, 8192), (1024, 8, 8192)]


@pytest.fixture(scope="module")
def big_batch_frames():
    frames = {}
    for name, insts in (("mix", BIG_MIX), ("same", BIG_SAME)):
        frames[name] = [rand_frame(120 + 10 * len(frames) + k, T, F, N)
                        for k, (N, F, T) in enumerate(insts)]
    ref = {name: [want(s) for s in fr] for name, fr in frames.items()}
    return frames, ref


@pytest.mark.parametrize("accumulate", [False, True])
def test_batch_more_tiles_than_slots(big_batch_frames, accumulate):
    frames, ref = big_batch_frames
    d = [torch.from_numpy(s).to(DEV) for s in frames["mix"]]
    rng = np.random.default_rng(130)
    starts = [rng.integers(-1_000_000, 1_000_000, engine.vis_shape(N, F)).astype(np.int32)
              if accumulate else np.full(engine.vis_shape(N, F), -7, np.int32)
              for N, F, T in BIG_MIX]
    vis = [torch.from_numpy(s).to(DEV) for s in starts]
    with BatchPlan(BIG_MIX, accumulate=accumulate) as bp:
        for rep in range(2):  # eager, then a graph replay
            if rep:
                for v, s in zip(vis, starts):
                    v.copy_(torch.from_numpy(s).to(DEV))
            bp.correlate(d, vis, graph=bool(rep))
            torch.cuda.synchronize()
            for k in range(len(BIG_MIX)):
                exp = ref["mix"][k] + (starts[k] if accumulate else 0)
                assert np.array_equal(vis[k].cpu().numpy(), exp), (rep, k)


def test_batch_more_tiles_than_slots_shared_vis(big_batch_frames):
    # two frames of one shape adding into one accumulator, as the request
    # loop's launches do
    frames, ref = big_batch_frames
    d = [torch.from_numpy(s).to(DEV) for s in frames["same"]]
    N, F, T = BIG_SAME[0]
    start = np.random.default_rng(131).integers(-1_000_000, 1_000_000,
                                                engine.vis_shape(N, F)).astype(np.int32)
    acc = torch.from_numpy(start).to(DEV)
    with BatchPlan(BIG_SAME, accumulate=True, shared_vis=True) as bp:
        bp.correlate(d, [acc, acc], graph=True)
        torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), ref["same"][0] + ref["same"][1] + start)
