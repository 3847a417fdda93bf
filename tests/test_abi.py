"""The C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before any HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1503_06202_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xeng.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xeng_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def test_version_and_strerror(L):
    assert L.xeng_version() >> 16 == 1
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.xeng_strerror(code)
    assert L.xeng_strerror(-99) == b"unknown error code"


def _plan(L, N, F, T, flags=0):
    h = ctypes.c_void_p()
    rc = L.xeng_plan(ctypes.byref(h), N, F, T, flags)
    return rc, h


def test_plan_validation(L):
    assert L.xeng_plan(None, 4, 1, 1, 0) == _lib.XENG_EINVAL
    for N, F, T in ((0, 1, 1), (1, 0, 1), (1, 1, 0), (-5, 1, 1), (_lib.XENG_N_MAX + 1, 1, 1)):
        rc, h = _plan(L, N, F, T)
        assert rc == _lib.XENG_EINVAL and not h.value
    rc, h = _plan(L, 4, 1, _lib.XENG_T_EXACT_MAX + 1)
    assert rc == _lib.XENG_EOVERFLOW
    for bad in (2, 0x200, 1 << 20, 0xFF):
        rc, h = _plan(L, 4, 1, 16, bad)
        assert rc == _lib.XENG_EINVAL, bad
    rc, h = _plan(L, _lib.XENG_N_MAX, 3, _lib.XENG_T_EXACT_MAX, _lib.XENG_FORM_F8 | _lib.XENG_ACCUMULATE)
    assert rc == _lib.XENG_OK and h.value
    assert L.xeng_destroy(h) == 0
    assert L.xeng_destroy(None) == 0


def test_correlate_validation_needs_no_gpu(L):
    rc, h = _plan(L, 64, 2, 1000)
    assert rc == 0
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
    try:
        assert L.xeng_correlate(None, dummy, 64, 2, 10, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate(h, None, 64, 2, 10, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate(h, dummy, 64, 2, 10, None, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate(h, dummy, 64, 2, 0, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate(h, dummy, 65, 2, 10, dummy, None) == _lib.XENG_EPLAN
        assert L.xeng_correlate(h, dummy, 64, 3, 10, dummy, None) == _lib.XENG_EPLAN
        assert L.xeng_correlate(h, dummy, 64, 2, 1001, dummy, None) == _lib.XENG_EPLAN
        assert L.xeng_correlate(h, dummy, 64, 2, 1 << 24, dummy, None) == _lib.XENG_EOVERFLOW
        assert L.xeng_plan_set_tuning(h, -1, 0) == _lib.XENG_EINVAL
        assert L.xeng_plan_set_tuning(h, 3, 6) == _lib.XENG_EINVAL
        assert L.xeng_plan_set_tuning(h, 3, -1) == _lib.XENG_EINVAL
        for k in (0, 1, 2, 3, 4, 5):
            assert L.xeng_plan_set_tuning(h, 3, k) == _lib.XENG_OK
        assert L.xeng_plan_error(h) == b""
    finally:
        L.xeng_destroy(h)


def test_gated_validation_needs_no_gpu(L):
    h = ctypes.c_void_p()
    # gate-count and shape errors are found before any allocation
    assert L.xeng_plan_gated(None, 64, 2, 1000, 4, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_gated(ctypes.byref(h), 64, 2, 1000, 0, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_gated(ctypes.byref(h), 64, 2, 1000, _lib.XENG_G_MAX + 1, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_gated(ctypes.byref(h), 0, 2, 1000, 4, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_gated(ctypes.byref(h), 64, 2, 1 << 24, 4, 0) == _lib.XENG_EOVERFLOW
    assert not h.value
    rc, hp = _plan(L, 64, 2, 1000)
    assert rc == 0
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced
    gate = (ctypes.c_int32 * 10)()
    try:
        assert L.xeng_correlate_gated(None, dummy, 64, 2, 10, gate, 2, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate_gated(hp, dummy, 64, 2, 10, None, 2, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate_gated(hp, dummy, 64, 2, 10, gate, 0, dummy, None) == _lib.XENG_EINVAL
        # a plan made by xeng_plan cannot gate
        assert L.xeng_correlate_gated(hp, dummy, 64, 2, 10, gate, 2, dummy, None) == _lib.XENG_EPLAN
    finally:
        L.xeng_destroy(hp)


def test_flagged_validation_needs_no_gpu(L):
    h = ctypes.c_void_p()
    assert L.xeng_plan_flagged(None, 64, 2, 1000, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_flagged(ctypes.byref(h), 0, 2, 1000, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_flagged(ctypes.byref(h), 64, 2, 1000, 1 << 12) == _lib.XENG_EINVAL
    assert L.xeng_plan_flagged(ctypes.byref(h), 64, 2, 1 << 24, 0) == _lib.XENG_EOVERFLOW
    assert not h.value
    rc, hp = _plan(L, 64, 2, 1000)
    assert rc == 0
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced
    try:
        f = L.xeng_correlate_flagged
        assert f(None, dummy, dummy, 64, 2, 10, dummy, dummy, None) == _lib.XENG_EINVAL
        assert f(hp, dummy, None, 64, 2, 10, dummy, dummy, None) == _lib.XENG_EINVAL
        assert f(hp, dummy, dummy, 64, 2, 10, dummy, None, None) == _lib.XENG_EINVAL
        assert f(hp, dummy, dummy, 64, 2, 0, dummy, dummy, None) == _lib.XENG_EINVAL
        # a plan made by xeng_plan has no count workspace
        assert f(hp, dummy, dummy, 64, 2, 10, dummy, dummy, None) == _lib.XENG_EPLAN
        n = L.xeng_normalize
        assert n(None, dummy, dummy, 1.0, dummy, None) == _lib.XENG_EINVAL
        assert n(hp, dummy, None, 1.0, dummy, None) == _lib.XENG_EINVAL
        assert n(hp, dummy, dummy, 0.0, dummy, None) == _lib.XENG_EINVAL
        assert n(hp, dummy, dummy, float("nan"), dummy, None) == _lib.XENG_EINVAL
        assert n(hp, dummy, dummy, float("inf"), dummy, None) == _lib.XENG_EINVAL
    finally:
        L.xeng_destroy(hp)


def test_beam_validation_needs_no_gpu(L):
    h = ctypes.c_void_p()
    assert L.xeng_plan_beams(None, 64, 2, 1000, 4, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_beams(ctypes.byref(h), 64, 2, 1000, 0, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_beams(ctypes.byref(h), 64, 2, 1000, _lib.XENG_BEAMS_MAX + 1, 0) == _lib.XENG_EINVAL
    assert L.xeng_plan_beams(ctypes.byref(h), 64, 2, 1000, 4, 1) == _lib.XENG_EINVAL
    assert L.xeng_plan_beams(ctypes.byref(h), 32768, 1024, 1000, 4, 0) == _lib.XENG_EINVAL
    assert not h.value
    rc, hp = _plan(L, 64, 2, 1000)
    assert rc == 0
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced
    try:
        w = (ctypes.c_int8 * 4)()
        assert L.xeng_beam_set_weights(None, w) == _lib.XENG_EINVAL
        assert L.xeng_beam_set_weights(hp, None) == _lib.XENG_EINVAL
        assert L.xeng_beam_set_weights(hp, w) == _lib.XENG_EPLAN       # not a beam plan
        assert L.xeng_beamform(None, dummy, 64, 2, 10, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_beamform(hp, dummy, 64, 2, 0, dummy, None) == _lib.XENG_EINVAL
        assert L.xeng_beamform(hp, dummy, 64, 2, 10, dummy, None) == _lib.XENG_EPLAN
    finally:
        L.xeng_destroy(hp)


def test_delay_validation_needs_no_gpu(L):
    rc, h = _plan(L, 40, 2, 1000)
    assert rc == 0
    D = (ctypes.c_int32 * 40)
    try:
        ok = D(*([5] * 16 + [0] * 16 + [9] * 8))
        assert L.xeng_plan_set_delays(None, ok, 10) == _lib.XENG_EINVAL
        assert L.xeng_plan_set_delays(h, ok, 8) == _lib.XENG_EINVAL        # 9 > D_max
        assert L.xeng_plan_set_delays(h, ok, -1) == _lib.XENG_EINVAL
        split = D(*([5] * 15 + [6] + [0] * 24))                          # differs within a group
        assert L.xeng_plan_set_delays(h, split, 10) == _lib.XENG_EINVAL
        assert L.xeng_plan_set_delays(h, ok, 1 << 30) == _lib.XENG_EINVAL  # offsets past 2^31
        assert L.xeng_plan_set_delays(h, None, 0) == _lib.XENG_OK           # off
    finally:
        L.xeng_destroy(h)
    arr = (_lib.XengInstance * 1)(_lib.XengInstance(8, 1, 8, 0))
    hb = ctypes.c_void_p()
    assert L.xeng_plan_batch(ctypes.byref(hb), arr, 1, 0) == 0
    try:
        assert L.xeng_plan_set_delays(hb, D(*([0] * 40)), 0) == _lib.XENG_EPLAN
    finally:
        L.xeng_destroy(hb)


def test_batch_validation_needs_no_gpu(L):
    def plan(descs, flags=0):
        arr = (_lib.XengInstance * len(descs))(*[_lib.XengInstance(*d) for d in descs])
        h = ctypes.c_void_p()
        return L.xeng_plan_batch(ctypes.byref(h), arr, len(descs), flags), h

    assert plan([(0, 1, 1, 0)])[0] == _lib.XENG_EINVAL
    assert plan([(8, 1, 1, -1)])[0] == _lib.XENG_EINVAL
    assert plan([(8, 1, 1 << 24, 0)])[0] == _lib.XENG_EOVERFLOW
    assert plan([(8, 1, 8, 0)], flags=7)[0] == _lib.XENG_EINVAL
    # shared outputs are atomic adds: only meaningful when accumulating
    assert plan([(8, 1, 8, 0)], flags=_lib.XENG_SHARED_VIS)[0] == _lib.XENG_EINVAL
    rc, hs = plan([(8, 1, 8, 0)], flags=_lib.XENG_SHARED_VIS | _lib.XENG_ACCUMULATE)
    assert rc == 0
    L.xeng_destroy(hs)
    # and single plans do not take the flag
    h1 = ctypes.c_void_p()
    assert L.xeng_plan(ctypes.byref(h1), 8, 1, 8, _lib.XENG_SHARED_VIS | _lib.XENG_ACCUMULATE) == _lib.XENG_EINVAL
    h = ctypes.c_void_p()
    assert L.xeng_plan_batch(ctypes.byref(h), None, 1, 0) == _lib.XENG_EINVAL
    rc, hb = plan([(64, 4, 8192, 0), (33, 1, 100, 3)])
    assert rc == 0 and hb.value
    dummy = ctypes.c_void_p(0x1000)
    try:
        both = (ctypes.c_void_p * 2)(dummy, dummy)
        half = (ctypes.c_void_p * 2)(dummy, None)
        # an active instance (non-NULL samples) needs its vis
        assert L.xeng_correlate_batch(hb, both, half, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate_batch(hb, None, both, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate_batch(hb, both, None, None) == _lib.XENG_EINVAL
        assert L.xeng_correlate_batch_graph(hb, both, half, None) == _lib.XENG_EINVAL
        # a single plan is not a batch plan, and the other way round
        rc, hs = _plan(L, 8, 1, 8)
        ok = (ctypes.c_void_p * 2)(dummy, dummy)
        assert L.xeng_correlate_batch(hs, ok, ok, None) == _lib.XENG_EPLAN
        assert L.xeng_correlate(hb, dummy, 64, 4, 10, dummy, None) == _lib.XENG_EPLAN
        L.xeng_destroy(hs)
    finally:
        L.xeng_destroy(hb)


def test_python_layer_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libxeng.so")
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_python_layer_rejects_cpu_tensors():
    import torch
    from paper_1503_06202_amd import engine
    with pytest.raises(ValueError):
        engine._check_samples(torch.zeros((4, 1, 8), dtype=torch.uint8))
    with pytest.raises(ValueError):
        engine._check_samples(torch.zeros((4, 8), dtype=torch.uint8))


def test_noalloc_batch_validation_needs_no_gpu(L):
    # argument errors and the fixed workspace's limits are decided on the host
    # before any HIP call
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced
    n = _lib.XENG_NOALLOC_INST_MAX + 1
    inst = (_lib.XengInstance * n)(*[_lib.XengInstance(16, 1, 64, 0)] * n)
    sp = (ctypes.c_void_p * n)(*[dummy] * n)
    vp = (ctypes.c_void_p * n)(*[dummy] * n)
    f = L.xeng_correlate_batch_noalloc
    assert f(None, 1, 0, sp, vp, None) == _lib.XENG_EINVAL
    assert f(inst, 0, 0, sp, vp, None) == _lib.XENG_EINVAL
    assert f(inst, 1, 0, None, vp, None) == _lib.XENG_EINVAL
    assert f(inst, 1, 0x400, sp, vp, None) == _lib.XENG_EINVAL
    assert f(inst, 1, _lib.XENG_SHARED_VIS, sp, vp, None) == _lib.XENG_EINVAL
    assert f(inst, n, 0, sp, vp, None) == _lib.XENG_ELIMIT
    bad = (_lib.XengInstance * 1)(_lib.XengInstance(16, 1, 64, -1))
    assert f(bad, 1, 0, sp, vp, None) == _lib.XENG_EINVAL
    big = (_lib.XengInstance * 1)(_lib.XengInstance(16, 1, _lib.XENG_T_EXACT_MAX + 1, 0))
    sp2 = (ctypes.c_void_p * 1)(dummy)
    vp2 = (ctypes.c_void_p * 1)(dummy)
    assert f(big, 1, 0, sp2, vp2, None) == _lib.XENG_EOVERFLOW
    # N = 32768: 32896 tiles per channel, so two channels are more work items
    # than the workspace holds
    many = (_lib.XengInstance * 1)(_lib.XengInstance(_lib.XENG_N_MAX, 2, 64, 0))
    assert f(many, 1, 0, sp2, vp2, None) == _lib.XENG_ELIMIT
    vnull = (ctypes.c_void_p * 1)()
    assert f(many, 1, 0, sp2, vnull, None) == _lib.XENG_EINVAL
