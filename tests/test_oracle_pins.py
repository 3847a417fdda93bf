"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import numpy as np
import pytest

import oracle
from oracle import build as obuild
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin, oracle_lib):
    pin(oracle_lib)


@pytest.mark.parametrize("pin", pins.SHIFT_PINS, ids=lambda p: p.__name__)
def test_shift_pin(pin, oracle_lib):
    pin(oracle_lib)


@pytest.mark.parametrize("mutant", obuild.SHIFT_MUTANTS + ("CONJ", "INDEX"))
def test_planted_shift_mistake_is_caught(mutant, tmp_path):
    """A copy of the oracle with a planted mistake fails at least one shift pin."""
    path = obuild.build(mutant, outdir=str(tmp_path))
    lib = oracle.load(path=path)
    failed = []
    for pin in pins.SHIFT_PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {mutant} passed every shift pin"


@pytest.mark.parametrize("pin", pins.FLAG_PINS, ids=lambda p: p.__name__)
def test_flag_pin(pin, oracle_lib):
    pin(oracle_lib)


@pytest.mark.parametrize("mutant", obuild.FLAG_MUTANTS + ("CONJ", "INDEX", "NIBBLE"))
def test_planted_flag_mistake_is_caught(mutant, tmp_path):
    """A copy of the oracle with a planted mistake fails at least one flag pin."""
    path = obuild.build(mutant, outdir=str(tmp_path))
    lib = oracle.load(path=path)
    failed = []
    for pin in pins.FLAG_PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {mutant} passed every flag pin"


@pytest.mark.parametrize("pin", pins.BEAM_PINS, ids=lambda p: p.__name__)
def test_beam_pin(pin, oracle_lib):
    pin(oracle_lib)


@pytest.mark.parametrize("mutant", obuild.BEAM_MUTANTS + ("NIBBLE", "OFFSET"))
def test_planted_beam_mistake_is_caught(mutant, tmp_path):
    """A copy of the oracle with a planted mistake fails at least one beam pin."""
    path = obuild.build(mutant, outdir=str(tmp_path))
    lib = oracle.load(path=path)
    failed = []
    for pin in pins.BEAM_PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {mutant} passed every beam pin"


@pytest.mark.parametrize("mutant", obuild.MUTANTS)
def test_planted_mistake_is_caught(mutant, tmp_path):
    """A copy of the oracle with one planted mistake fails at least one pin."""
    path = obuild.build(mutant, outdir=str(tmp_path))
    lib = oracle.load(path=path)
    failed = []
    for pin in pins.FAST_PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutant {mutant} passed every pin"


def test_gated_sums_to_ungated(oracle_lib):
    """Output gating: the gate buffers partition the integration (Sec. IV-C, Output Gating)."""
    rng = np.random.default_rng(3)
    T, F, N, G = 97, 2, 6, 3
    s = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    gate = rng.integers(0, G, T)
    g = oracle.correlate_gated(s, gate, G, lib=oracle_lib)
    assert np.array_equal(g.sum(axis=0), oracle.correlate(s, lib=oracle_lib))
    # each gate alone equals the ungated oracle on that gate's samples only
    for k in range(G):
        sel = s[gate == k]
        assert np.array_equal(g[k], oracle.correlate(sel, lib=oracle_lib))
    # samples with a gate outside [0, G) go nowhere
    gate2 = gate.copy()
    gate2[::5] = -1
    g2 = oracle.correlate_gated(s, gate2, G, lib=oracle_lib)
    assert np.array_equal(g2.sum(axis=0), oracle.correlate(s[gate2 >= 0], lib=oracle_lib))


def test_to_int32_refuses_overflow():
    with pytest.raises(OverflowError):
        oracle.to_int32(np.array([2 ** 31], dtype=np.int64))
    assert oracle.to_int32(np.array([2 ** 31 - 1], dtype=np.int64))[0] == 2 ** 31 - 1


def test_tri_index_matches_triu_order():
    N = 9
    iu, ju = np.triu_indices(N)
    assert [oracle.tri_index(int(i), int(j), N) for i, j in zip(iu, ju)] == list(range(len(iu)))


def test_pairs_agree_with_full(oracle_lib):
    """The one-baseline-at-a-time entry equals the full-channel result (both orders of i, j)."""
    rng = np.random.default_rng(4)
    T, F, N = 77, 3, 11
    s = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    full = oracle.correlate(s, full=True, lib=oracle_lib)
    f = rng.integers(0, F, 200)
    i = rng.integers(0, N, 200)
    j = rng.integers(0, N, 200)
    got = oracle.correlate_pairs(s, f, i, j, lib=oracle_lib)
    assert np.array_equal(got, full[f, i, j])
