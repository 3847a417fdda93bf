"""The streaming loop and the autotuner on the GPU (parity with the oracle)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1503_06202_amd import BatchPlan, Plan, tune, vis_shape
from paper_1503_06202_amd.stream import Frame, GpuLauncher, RequestLoop, poisson_arrivals

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph,queues,tuned", [(False, 1, False), (True, 1, False),
                                                (True, 2, False), (True, 1, True)])
def test_request_loop_accumulates_exactly(graph, queues, tuned):
    # one HIP stream with two launches queued (the default), or launches on
    # two HIP streams adding into the same accumulators; with slices tuned
    # per batch size or the library's automatic count
    N, F, T, streams = 136, 2, 320, 3
    rng = np.random.default_rng(17)
    host = [rng.integers(0, 256, (T, F, N), dtype=np.uint8) for _ in range(12)]
    pool = [torch.from_numpy(h).cuda() for h in host]
    n = 40
    arr = poisson_arrivals(n, 4000.0, 5)
    frames = [Frame(k, k % streams, pool[k % len(pool)], float(arr[k])) for k in range(n)]
    la = GpuLauncher(N, F, T, slots=4, streams=streams, graph=graph, max_batch=4,
                     dump_buffers=16, queues=queues)
    if tuned:
        choice = la.tune_slices(pool[:4], candidates=(0, 1, 2, 3))
        assert set(choice) == {1, 2, 3, 4} and set(choice.values()) <= {0, 1, 2, 3}
        assert all(float(la.acc[st].abs().sum()) == 0 for st in range(streams))  # untouched
    rep = RequestLoop(la, dump_every=5).run(frames)
    torch.cuda.synchronize()
    assert rep.frames == n and max(rep.batch_sizes) <= 4
    for st in range(streams):
        want = sum(oracle.correlate(host[k % len(host)]) for k in range(n) if k % streams == st)
        dumped = [d for s, c, d in rep.dumps if s == st]
        got = sum(h.numpy().astype(np.int64) for (_, h, _) in dumped) + la.acc[st].cpu().numpy()
        assert np.array_equal(got, want), st
    la.close()


def test_checkpoint_restore_resume_is_bit_identical():
    # an integration checkpointed after 7 frames and resumed in a new launcher
    # (fresh plans and accumulators) dumps exactly what an uninterrupted run
    # dumps, and ends with the same pending sums
    N, F, T, n = 136, 2, 320, 15
    rng = np.random.default_rng(19)
    host = [rng.integers(0, 256, (T, F, N), dtype=np.uint8) for _ in range(n)]
    dev = [torch.from_numpy(h).cuda() for h in host]
    arr = poisson_arrivals(n, 3000.0, 7)

    def frames(lo, hi):
        return [Frame(k, 0, dev[k], float(arr[k] - arr[lo])) for k in range(lo, hi)]

    def run(la, fr, since=None):
        rep = RequestLoop(la, dump_every=4).run(fr, since_dump=since)
        torch.cuda.synchronize()
        return rep, [(c, h.numpy().copy()) for (_, c, (_, h, _)) in rep.dumps]

    la = GpuLauncher(N, F, T, slots=6, max_batch=3, dump_buffers=8)
    rep, whole = run(la, frames(0, n))
    whole_acc = la.acc[0].cpu().numpy()
    la.close()

    la1 = GpuLauncher(N, F, T, slots=6, max_batch=3, dump_buffers=8)
    rep1, part1 = run(la1, frames(0, 7))
    state, since = la1.checkpoint(), dict(rep1.pending)
    la1.close()
    la2 = GpuLauncher(N, F, T, slots=6, max_batch=3, dump_buffers=8)
    la2.restore(state)
    rep2, part2 = run(la2, frames(7, n), since)
    resumed_acc = la2.acc[0].cpu().numpy()
    la2.close()
    assert [c for c, _ in part1 + part2] == [c for c, _ in whole]
    for (_, a), (_, b) in zip(part1 + part2, whole):
        assert np.array_equal(a, b)
    assert np.array_equal(resumed_acc, whole_acc)
    # and the dumps are the oracle's sums over their frames
    assert np.array_equal(whole[0][1], oracle.to_int32(sum(oracle.correlate(h) for h in host[:4])))


def test_alone_equals_share_in_mix():
    # each frame alone (plain plan) equals what it adds to its stream's accumulator
    N, F, T = 200, 1, 256
    rng = np.random.default_rng(3)
    fr = [torch.from_numpy(rng.integers(0, 256, (T, F, N), dtype=np.uint8)).cuda() for _ in range(5)]
    with Plan(N, F, T) as p:
        alone = [p.correlate(x).clone() for x in fr]
    acc = torch.zeros(vis_shape(N, F), dtype=torch.int32, device="cuda")
    with BatchPlan([(N, F, T)] * 5, accumulate=True, shared_vis=True) as bp:
        bp.correlate(fr, [acc] * 5)
        torch.cuda.synchronize()
        assert torch.equal(acc, sum(alone))
        # a subset of slots: the others are skipped and add nothing
        acc2 = torch.zeros_like(acc)
        bp.correlate([fr[0], None, fr[2], None, None], [acc2, None, acc2, None, None], graph=True)
        torch.cuda.synchronize()
        assert torch.equal(acc2, alone[0] + alone[2])


def test_tuner_choices_are_exact(tmp_path):
    insts = [(64, 2, 1024)] * 3 + [(130, 1, 512), (256, 2, 2048)]
    path = str(tmp_path / "tune.json")
    splits = tune.tune(insts, cache_path=path, reps=2)
    assert len(splits) == len(insts) and all(s in tune.CANDIDATES for s in splits)
    # the cache is reused
    assert tune.tune(insts, cache_path=path, reps=2) == splits
    rng = np.random.default_rng(8)
    host = [rng.integers(0, 256, (T, F, N), dtype=np.uint8) for N, F, T in insts]
    d = [torch.from_numpy(h).cuda() for h in host]
    vis = [torch.empty(vis_shape(N, F), dtype=torch.int32, device="cuda") for N, F, T in insts]
    with BatchPlan(insts, split_t=splits) as bp:
        bp.correlate(d, vis, graph=True)
        torch.cuda.synchronize()
    for h, v in zip(host, vis):
        assert np.array_equal(v.cpu().numpy(), oracle.to_int32(oracle.correlate(h)))


@pytest.mark.parametrize("N,F,T", [(384, 4, 2048), (200, 8, 4096)])
def test_plain_tuner_picks_an_exact_tile_shape(tmp_path, N, F, T):
    # at N <= 256 the channel kernel (kernel 5) is among the timed candidates
    path = str(tmp_path / "tune.json")
    kernel, split = tune.tune_plain(N, F, T, reps=2, cache_path=path)
    assert kernel in tune.PLAIN_KERNELS and split in tune.PLAIN_SPLITS
    assert tune.tune_plain(N, F, T, reps=2, cache_path=path) == (kernel, split)  # cached
    timed = {k.split("/")[0] for k in next(iter(tune.load_cache(path).values()))["ms"]}
    assert ("5" in timed) == (N <= 256)
    s = np.random.default_rng(9).integers(0, 256, (T, F, N), dtype=np.uint8)
    with Plan(N, F, T, split_t=split, kernel=kernel) as p:
        got = p.correlate(torch.from_numpy(s).cuda()).cpu().numpy()
    assert np.array_equal(got, oracle.to_int32(oracle.correlate(s)))
