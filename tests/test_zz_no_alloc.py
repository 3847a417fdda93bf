"""The allocation-free batched entry point (``xeng_correlate_batch_noalloc``)
against the planned batched form (``xeng_plan_batch`` +
``xeng_correlate_batch``) and the oracle, through the C ABI.

Two calls in a row share the library's fixed workspace; the second has fewer
and smaller instances, so a stale work list or instance table from the first
call would show in its output.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1503_06202_amd import BatchPlan, engine

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")

FIRST = [(1, 1, 64), (17, 2, 100), (64, 4, 1000), (130, 1, 257), (256, 2, 640), (9, 3, 7),
         (300, 1, 2000), (64, 1, 64), (2048, 1, 1024)]
SECOND = [(40, 1, 300), (200, 2, 130), (5, 1, 9)]


def frames(instances, seed):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, 256, (T, F, N), dtype=np.uint8) for N, F, T in instances]


def new_vis(instances, fill=-7):
    return [torch.full(engine.vis_shape(N, F), fill, dtype=torch.int32, device=DEV)
            for N, F, T in instances]


def planned(instances, d, form, split_t=None):
    vis = new_vis(instances)
    with BatchPlan(instances, form=form, split_t=split_t) as bp:
        bp.correlate(d, vis)
        torch.cuda.synchronize()
    return [v.cpu().numpy() for v in vis]


@pytest.mark.parametrize("form", ["i8", "f8"])
@pytest.mark.parametrize("splits", [None, [1, 2, 3, 1, 4, 1, 2, 5, 2]])
def test_noalloc_matches_planned_batch(form, splits):
    hs = [frames(FIRST, 71), frames(SECOND, 72)]
    for call, (inst, h) in enumerate(zip((FIRST, SECOND), hs)):
        print(f"noalloc call {call} form={form} splits={splits} instances={len(inst)}", flush=True)
        d = [torch.from_numpy(x).to(DEV) for x in h]
        sp = splits[:len(inst)] if splits else None
        vis = new_vis(inst)
        engine.correlate_batch_noalloc(inst, d, vis, form=form, split_t=sp)
        torch.cuda.synchronize()
        ref = planned(inst, d, form, sp)
        for k, x in enumerate(h):
            got = vis[k].cpu().numpy()
            assert np.array_equal(got, ref[k]), (call, k)
            assert np.array_equal(got, oracle.to_int32(oracle.correlate(x))), (call, k)


def test_noalloc_skips_and_accumulates():
    h = frames(SECOND, 73)
    d = [torch.from_numpy(x).to(DEV) for x in h]
    vis = new_vis(SECOND, fill=5)
    engine.correlate_batch_noalloc(SECOND, [d[0], None, d[2]], [vis[0], None, vis[2]],
                                   accumulate=True)
    torch.cuda.synchronize()
    for k in (0, 2):
        want = oracle.to_int32(oracle.correlate(h[k])) + 5
        assert np.array_equal(vis[k].cpu().numpy(), want), k
    assert (vis[1].cpu().numpy() == 5).all()  # skipped: untouched
