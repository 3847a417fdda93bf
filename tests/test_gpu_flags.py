"""Flagged data on the GPU against the oracle's flagged definition (Sec. IV-A,
"Data Flow"): a flagged sample takes no part in the integration, and every
baseline carries the number of times both of its inputs were valid.

Expected values come from the oracle (``oracle.correlate_flagged`` and
``oracle.normalize``) on the same seeded bytes and flag words.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1503_06202_amd import Plan

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def rand_frame(seed, T, F, N):
    return np.random.default_rng(seed).integers(0, 256, (T, F, N), dtype=np.uint8)


def rand_invalid(seed, T, F, N, p, rows=0.0, junk_bits=True):
    """Random invalid samples with probability p, plus whole rows (all inputs
    of one (t, f)) with probability ``rows``; flag words with junk in the bits
    of inputs >= N when ``junk_bits``."""
    rng = np.random.default_rng(seed)
    inv = rng.random((T, F, N)) < p
    if rows:
        inv |= (rng.random((T, F)) < rows)[:, :, None]
    fl = synth.pack_flags(inv)
    if junk_bits and N % 32:
        junk = rng.integers(0, 2**32, fl.shape[:2], dtype=np.uint64).astype(np.uint32)
        fl[:, :, -1] |= junk & np.uint32(~((1 << (N % 32)) - 1) & 0xFFFFFFFF)
    return inv, fl


def gpu_flagged(s, fl, form="i8", vis=None, counts=None, accumulate=False, plan=None):
    T, F, N = s.shape
    d = torch.from_numpy(np.ascontiguousarray(s)).to(DEV)
    f = torch.from_numpy(np.ascontiguousarray(fl).view(np.int32)).to(DEV)
    own = plan is None
    p = plan or Plan(N, F, T, form=form, accumulate=accumulate, flagged=True)
    try:
        v, c = p.correlate_flagged(d, f, vis, counts)
        torch.cuda.synchronize()
        return v.cpu().numpy(), c.cpu().numpy(), d.cpu().numpy()
    finally:
        if own:
            p.close()


def want(s, fl):
    v, c = oracle.correlate_flagged(s, fl)
    return oracle.to_int32(v), oracle.to_int32(c)


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("N,T", [(96, 300), (40, 129), (128, 1000)])
def test_flagged_matches_oracle(form, N, T):
    F = 3
    s = rand_frame(101 + N, T, F, N)
    inv, fl = rand_invalid(102 + N, T, F, N, 0.05, rows=0.02)
    print(f"flagged N={N} T={T} F={F} form={form}", flush=True)
    v, c, _ = gpu_flagged(s, fl, form)
    wv, wc = want(s, fl)
    assert np.array_equal(c, wc)
    assert np.array_equal(v, wv)


def test_no_flags_is_plain_correlation():
    T, F, N = 777, 2, 64
    s = rand_frame(103, T, F, N)
    fl = np.zeros((T, F, 2), np.uint32)
    v, c, s2 = gpu_flagged(s, fl)
    assert (c == T).all()
    assert np.array_equal(v, oracle.to_int32(oracle.correlate(s)))
    assert np.array_equal(s2, s)


def test_all_flagged_is_zero():
    T, F, N = 200, 2, 48
    s = rand_frame(104, T, F, N)
    fl = synth.pack_flags(np.ones((T, F, N), bool))
    v, c, s2 = gpu_flagged(s, fl)
    assert not v.any() and not c.any()
    assert (s2 == 0x88).all()


def test_samples_zeroed_in_place():
    T, F, N = 150, 2, 70
    s = rand_frame(105, T, F, N)
    inv, fl = rand_invalid(106, T, F, N, 0.2)
    _, _, s2 = gpu_flagged(s, fl)
    assert (s2[inv] == 0x88).all()
    assert np.array_equal(s2[~inv], s[~inv])


def test_single_and_multi_rows():
    """Rows with exactly one invalid input (counted apart) next to rows with
    several (correlated as events), in every position of a 64-row block."""
    T, F, N = 64 * 5 + 7, 2, 96
    s = rand_frame(107, T, F, N)
    rng = np.random.default_rng(108)
    inv = np.zeros((T, F, N), bool)
    for t in range(T):
        for f in range(F):
            k = int(rng.integers(0, 4))     # 0, 1, 2 or 3 invalid inputs
            inv[t, f, rng.choice(N, k, replace=False)] = True
    inv[10:50, 0, 5] = True                  # one input out for a stretch
    fl = synth.pack_flags(inv)
    v, c, _ = gpu_flagged(s, fl)
    wv, wc = want(s, fl)
    assert np.array_equal(c, wc)
    assert np.array_equal(v, wv)


@pytest.mark.parametrize("recipe", ["pathfinder", "heavy"])
def test_recipes(recipe):
    T, F, N = 4096, 2, 256
    s = synth.gen_frame(N, F, T, 9, "gauss")
    fl = synth.gen_flags(T, F, N, 10, recipe, link_channels=1)
    v, c, _ = gpu_flagged(s, fl)
    wv, wc = want(s, fl)
    assert np.array_equal(c, wc)
    assert np.array_equal(v, wv)


def test_repeated_patterns_of_every_length():
    """Runs of identical rows (one invalid set repeated m times, m = 1..64)
    inside and across 64-row blocks: every group size has its own weights."""
    T, F, N = 64 * 70, 2, 100
    s = rand_frame(120, T, F, N)
    rng = np.random.default_rng(121)
    inv = np.zeros((T, F, N), bool)
    t = 0
    for m in list(range(1, 65)) + [100, 3, 130, 2]:
        if t >= T:
            break
        for f in range(F):
            inv[t:t + m, f, :] = rng.random(N) < (0.02 if f else 0.3)
        t += m
    fl = synth.pack_flags(inv)
    v, c, _ = gpu_flagged(s, fl)
    wv, wc = want(s, fl)
    assert np.array_equal(c, wc)
    assert np.array_equal(v, wv)


def test_event_rows_span_two_launch_segments():
    """Every row has its own set of several invalid inputs, so the event frame
    holds more rows than one int8 launch may integrate (2^19) and is
    correlated in two launches."""
    T, F, N = (1 << 20) + 4096, 1, 32
    s = rand_frame(109, T, F, N)
    rng = np.random.default_rng(110)
    fl = rng.integers(0, 2**32, (T, F, 1), dtype=np.uint64).astype(np.uint32)
    fl[np.bitwise_count(fl) < 2] = 3
    print(f"flagged segments T={T}", flush=True)
    v, c, _ = gpu_flagged(s, fl)
    wv, wc = want(s, fl)
    assert np.array_equal(c, wc)
    assert np.array_equal(v, wv)


def test_accumulate_adds_vis_and_counts():
    T, F, N = 500, 2, 64
    s1, s2 = rand_frame(111, T, F, N), rand_frame(112, T, F, N)
    _, f1 = rand_invalid(113, T, F, N, 0.1, rows=0.05)
    _, f2 = rand_invalid(114, T, F, N, 0.1, rows=0.05)
    w1, c1 = want(s1, f1)
    w2, c2 = want(s2, f2)
    with Plan(N, F, T, accumulate=True, flagged=True) as p:
        vis = torch.from_numpy(np.full(w1.shape, 5, np.int32)).to(DEV)
        cnt = torch.from_numpy(np.full(c1.shape, -2, np.int32)).to(DEV)
        gpu_flagged(s1, f1, vis=vis, counts=cnt, plan=p)
        v, c, _ = gpu_flagged(s2, f2, vis=vis, counts=cnt, plan=p)
    assert np.array_equal(v, w1 + w2 + 5)
    assert np.array_equal(c, c1 + c2 - 2)


def test_plan_reuse_shrinking_events():
    """A second call with fewer event rows must not see the first call's."""
    T, F, N = 900, 2, 64
    with Plan(N, F, T, flagged=True) as p:
        for seed, rows in ((115, 0.5), (116, 0.0), (117, 0.01)):
            s = rand_frame(seed, T, F, N)
            _, fl = rand_invalid(seed + 50, T, F, N, 0.01 if rows else 0.0, rows=rows)
            v, c, _ = gpu_flagged(s, fl, plan=p)
            wv, wc = want(s, fl)
            assert np.array_equal(c, wc), seed
            assert np.array_equal(v, wv), seed


@pytest.mark.parametrize("scale", [1.0, 4096.0, 3.7])
def test_normalize_matches_oracle(scale):
    T, F, N = 4096, 2, 80
    s = synth.gen_frame(N, F, T, 11, "gauss")
    _, fl = rand_invalid(118, T, F, N, 0.1, rows=0.01)
    fl[:, 1, 0] = 0xFFFFFFFF                       # channel 1: inputs 0..31 never valid
    d = torch.from_numpy(s).to(DEV)
    f = torch.from_numpy(fl.view(np.int32)).to(DEV)
    with Plan(N, F, T, flagged=True) as p:
        v, c = p.correlate_flagged(d, f)
        out = p.normalize(v, c, scale)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    wv, wc = oracle.correlate_flagged(s, fl)
    ref = oracle.normalize(wv, wc, scale)
    assert (wc == 0).any()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_flagged_needs_no_shift():
    from paper_1503_06202_amd import _lib

    T, F, N = 64, 1, 32
    s = torch.zeros((T, F, N), dtype=torch.uint8, device=DEV)
    f = torch.zeros((T, F, 1), dtype=torch.int32, device=DEV)
    with Plan(N, F, T, flagged=True) as p:
        p.set_delays(np.zeros(N, np.int32), 4)
        with pytest.raises(_lib.XengError):
            p.correlate_flagged(s, f)
        p.set_delays(None)
        v, c = p.correlate_flagged(s, f)
        torch.cuda.synchronize()
        assert (c.cpu().numpy() == T).all()


def test_full_array_pathfinder_flags_subset():
    """The full-array frame (N=2048, F=16, T=32768) with the pathfinder flag
    recipe: counts and visibilities of all pairs among 48 sampled inputs in
    three channels against the oracle on that subset, and the counts'
    diagonal everywhere against the flag words."""
    w = synth.workload("full_array")
    s = synth.gen_frame(w.N, w.F, w.T, w.seed, w.kind)
    fl = synth.gen_flags(w.T, w.F, w.N, 12, "pathfinder")
    print(f"full_array flagged N={w.N} F={w.F} T={w.T}", flush=True)
    v, c, s2 = gpu_flagged(s, fl)
    rng = np.random.default_rng(119)
    idx = np.sort(rng.choice(w.N, 48, replace=False))
    for f in (0, 7, 15):
        sub = np.ascontiguousarray(s[:, f:f + 1, idx])
        inv = synth.unpack_flags(fl[:, f:f + 1, :], w.N)[:, :, idx]
        wv, wc = want(sub, synth.pack_flags(inv))
        ii, jj = np.triu_indices(len(idx))
        b = idx[ii] * w.N - idx[ii] * (idx[ii] - 1) // 2 + (idx[jj] - idx[ii])
        assert np.array_equal(c[f, b], wc[0]), f
        assert np.array_equal(v[f, b], wv[0]), f
    inv_count = np.zeros((w.F, w.N), np.int64)
    for t0 in range(0, w.T, 4096):
        inv_count += synth.unpack_flags(fl[t0:t0 + 4096], w.N).sum(axis=0)
    d = np.arange(w.N) * w.N - np.arange(w.N) * (np.arange(w.N) - 1) // 2
    assert np.array_equal(c[:, d], w.T - inv_count)
