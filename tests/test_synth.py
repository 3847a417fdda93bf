"""The seeded input generator: determinism, per-channel regeneration, value range."""
import numpy as np

import synth


def test_deterministic_sha():
    a = synth.gen_frame(64, 3, 1500, 7, "gauss+tone")
    b = synth.gen_frame(64, 3, 1500, 7, "gauss+tone")
    assert synth.frame_sha256(a) == synth.frame_sha256(b)
    c = synth.gen_frame(64, 3, 1500, 8, "gauss+tone")
    assert synth.frame_sha256(a) != synth.frame_sha256(c)


def test_channel_regeneration_and_prefix():
    a = synth.gen_frame(48, 5, 2100, 3, "gauss+tone")
    for f in range(5):
        assert np.array_equal(a[:, f, :], synth.gen_channel(48, 2100, 3, f, "gauss+tone", F=5))
    sub = synth.gen_frame(48, 5, 2100, 3, "gauss+tone", channels=[4, 1])
    assert np.array_equal(sub[:, 0], a[:, 4]) and np.array_equal(sub[:, 1], a[:, 1])
    short = synth.gen_frame(48, 5, 700, 3, "gauss+tone")
    assert np.array_equal(short, a[:700])


def test_value_range_and_stats():
    a = synth.gen_frame(128, 2, 4096, 2, "gauss")
    hi = (a >> 4).astype(int) - 8
    lo = (a & 15).astype(int) - 8
    for p in (hi, lo):
        assert p.min() >= -8 and p.max() <= 7
        assert 2.5 < p.std() < 5.0
    u = synth.gen_frame(16, 1, 256, 1, "uniform")
    assert set(np.unique(u >> 4)) <= set(range(16))


def test_encode_rejects_out_of_range():
    import pytest
    with pytest.raises(ValueError):
        synth.encode(np.array([8]), np.array([0]))


def test_tone_channels_count():
    from synth.frames import _tones
    assert len(_tones(3, 16, 8)) == 1
    assert len(_tones(3, 64, 8)) == 4


def test_batch_instances_seeded():
    a = synth.batch_instances()
    assert len(a) == 48 and a == synth.batch_instances()
    assert all(n in synth.frames.N_CHOICES and t in synth.frames.T_CHOICES and f == 4 for n, f, t in a)
