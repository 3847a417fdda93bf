"""Seeded synthetic sample frames in the F-engine's 4+4-bit offset format.

Layout of a frame: ``samples[T][F][N]`` uint8, where T is time, F frequency
channel and N the input (antenna feed).  One byte carries one complex sample:
the high nibble holds the real part and the low nibble the imaginary part, each
stored offset-binary, i.e. value + 8 so that [-8, 7] maps to [0, 15] (Sec. II-A,
footnote on the encoding).

Recipes (all draws from numpy PCG64 seeded through ``SeedSequence``):

* ``uniform``: real and imaginary parts i.i.d. uniform over the 16 values
  [-8, 7].
* ``gauss``: per component ``clip(rint(2.5 * (g_common[t] * a_i + g_indep[t, i])), -8, 7)``
  where ``g_common`` and ``g_indep`` are complex Gaussians with N(0, 1) real and
  imaginary parts and ``a_i`` a per-input gain uniform in [0.5, 1.5].  This
  gives inputs that are about 50% correlated with each other, with mild
  clipping, the statistics of a sky-noise dominated array.
* ``gauss+tone``: as ``gauss``, and ``ceil(5% of F)`` channels (chosen by seed)
  also carry a narrowband tone of amplitude 6, ``6 * exp(i (2 pi nu0 t + phi_i))``,
  added before rounding, with a seeded frequency ``nu0`` and per-input phase
  ``phi_i``: the strongly correlated case, like RFI or a bright source.

Every channel has its own random stream, so one channel can be regenerated
alone and equals the matching slice of the whole frame.  Draws proceed in
blocks of ``_TBLOCK`` time samples, so a frame of T samples is a prefix of any
longer frame with the same seed.
"""

from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import hashlib
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_TBLOCK = 1024          # time samples per draw block (fixes the stream layout)
_KEY_GAIN = 0xA11       # spawn keys for the per-instance draws
_KEY_TONE = 0x70E
_KEY_STREAM = 0x5EA
_KEY_BATCH = 0xBA7


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named synthetic workload: shape, recipe and seed."""

    name: str
    N: int
    F: int
    T: int
    kind: str
    seed: int
    note: str = ""

    @property
    def baselines(self) -> int:
        return self.N * (self.N + 1) // 2

    @property
    def cmac(self) -> int:
        """Useful complex multiply-accumulates of one frame, F * T * N(N+1)/2."""
        return self.F * self.T * self.baselines


WORKLOADS: Dict[str, Workload] = {
    w.name: w
    for w in (
        Workload("tiny", 16, 1, 256, "uniform", 1,
                 "N=16 inputs, 1 channel, 256 samples, uniform codes"),
        Workload("pathfinder", 256, 64, 32768, "gauss", 2,
                 "N=256 (the Pathfinder's 256 inputs), 64 channels, 32768 samples"),
        Workload("full_array", 2048, 16, 32768, "gauss+tone", 3,
                 "N=2048 (full-array inputs), 16 channels, 32768 samples, 5% toned channels"),
        Workload("precision", 2048, 16, 131072, "gauss+tone", 4,
                 "N=2048, 16 channels, 131072 samples (the FP8 form's workload)"),
        Workload("stream_frame", 2048, 4, 32768, "gauss", 5,
                 "one frame of the streaming loop: N=2048, 4 channels, 32768 samples"),
    )
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def encode(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Pack signed parts in [-8, 7] into offset-binary bytes (re high, im low)."""
    re = np.asarray(re, dtype=np.int16)
    im = np.asarray(im, dtype=np.int16)
    if re.size and (re.min() < -8 or re.max() > 7 or im.min() < -8 or im.max() > 7):
        raise ValueError("sample parts must lie in [-8, 7]")
    return (((re + 8) << 4) | (im + 8)).astype(np.uint8)


def _seq(seed: int, *key: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(int(seed), spawn_key=tuple(int(k) for k in key))


def _gains(seed: int, N: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(_seq(seed, _KEY_GAIN)))
    return rng.uniform(0.5, 1.5, size=N).astype(np.float32)


def _tones(seed: int, F: int, N: int) -> Dict[int, Tuple[float, np.ndarray]]:
    """Channels that carry a tone, with the tone's frequency and per-input phase."""
    rng = np.random.Generator(np.random.PCG64(_seq(seed, _KEY_TONE)))
    count = math.ceil(0.05 * F)
    chans = rng.choice(F, size=count, replace=False)
    out = {}
    for c in sorted(int(x) for x in chans):
        nu0 = float(rng.uniform(0.01, 0.49))
        phi = rng.uniform(0.0, 2.0 * math.pi, size=N)
        out[c] = (nu0, phi)
    return out


def gen_channel(N: int, T: int, seed: int, f: int, kind: str, F: Optional[int] = None,
                stream_key: Sequence[int] = ()) -> np.ndarray:
    """Samples of channel ``f`` alone, shape ``[T][N]`` uint8.

    ``F`` (the frame's channel count) is needed by ``gauss+tone`` to know which
    channels carry the tone.  ``stream_key`` separates independent frames that
    share a seed (the streaming loop's frame index).
    """
    if N < 1 or T < 0:
        raise ValueError("N >= 1 and T >= 0 required")
    rng = np.random.Generator(np.random.PCG64(_seq(seed, *stream_key, f)))
    out = np.empty((T, N), dtype=np.uint8)
    nblk = (T + _TBLOCK - 1) // _TBLOCK
    if kind == "uniform":
        for b in range(nblk):
            v = rng.integers(-8, 8, size=(_TBLOCK, N, 2), dtype=np.int16)
            t0 = b * _TBLOCK
            n = min(_TBLOCK, T - t0)
            out[t0:t0 + n] = encode(v[:n, :, 0], v[:n, :, 1])
        return out
    if kind not in ("gauss", "gauss+tone"):
        raise ValueError(f"unknown recipe {kind!r}")
    a = _gains(seed, N)
    tone = None
    if kind == "gauss+tone":
        if F is None:
            raise ValueError("gauss+tone needs F")
        tone = _tones(seed, F, N).get(f)
    for b in range(nblk):
        gc = rng.standard_normal((_TBLOCK, 1, 2), dtype=np.float32)
        gi = rng.standard_normal((_TBLOCK, N, 2), dtype=np.float32)
        t0 = b * _TBLOCK
        n = min(_TBLOCK, T - t0)
        x = gc[:n] * a[None, :, None]
        x += gi[:n]
        x *= np.float32(2.5)
        if tone is not None:
            nu0, phi = tone
            t = np.arange(t0, t0 + n, dtype=np.float64)[:, None]
            ang = 2.0 * math.pi * nu0 * t + phi[None, :]
            x[:, :, 0] += (6.0 * np.cos(ang)).astype(np.float32)
            x[:, :, 1] += (6.0 * np.sin(ang)).astype(np.float32)
        np.rint(x, out=x)
        np.clip(x, -8, 7, out=x)
        v = x.astype(np.int16)
        out[t0:t0 + n] = encode(v[:, :, 0], v[:, :, 1])
    return out


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def gen_frame(N: int, F: int, T: int, seed: int, kind: str,
              channels: Optional[Sequence[int]] = None, stream_key: Sequence[int] = (),
              out: Optional[np.ndarray] = None, threads: Optional[int] = None) -> np.ndarray:
    """A frame ``[T][len(channels)][N]`` uint8 (all F channels by default).

    Channels are generated on a thread pool; numpy's bulk draws release the
    interpreter lock, so this scales with host cores.
    """
    chans = list(range(F)) if channels is None else [int(c) for c in channels]
    for c in chans:
        if not 0 <= c < F:
            raise ValueError(f"channel {c} outside [0, {F})")
    if out is None:
        out = np.empty((T, len(chans), N), dtype=np.uint8)
    elif out.shape != (T, len(chans), N) or out.dtype != np.uint8:
        raise ValueError("out has the wrong shape or dtype")

    def one(k_c):
        k, c = k_c
        out[:, k, :] = gen_channel(N, T, seed, c, kind, F=F, stream_key=stream_key)

    nt = threads or _threads()
    if nt == 1 or len(chans) == 1:
        for kc in enumerate(chans):
            one(kc)
    else:
        with _cf.ThreadPoolExecutor(max_workers=nt) as ex:
            list(ex.map(one, enumerate(chans)))
    return out


def frame_sha256(samples: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(samples).tobytes()).hexdigest()


def stream_frame(k: int, w: Workload = WORKLOADS["stream_frame"], T: Optional[int] = None,
                 channels: Optional[Sequence[int]] = None) -> np.ndarray:
    """Frame ``k`` of the streaming loop (independent seeded draws per frame)."""
    return gen_frame(w.N, w.F, w.T if T is None else T, w.seed, w.kind,
                     channels=channels, stream_key=(_KEY_STREAM, k))


N_CHOICES = (64, 128, 256, 512, 1024, 2048)
T_CHOICES = (8192, 16384, 32768)


def batch_instances(count: int = 48, seed: int = 5, F: int = 4) -> List[Tuple[int, int, int]]:
    """(N, F, T) of the batched workload: N and T drawn uniformly from fixed sets."""
    rng = np.random.Generator(np.random.PCG64(_seq(seed, _KEY_BATCH)))
    Ns = rng.choice(N_CHOICES, size=count)
    Ts = rng.choice(T_CHOICES, size=count)
    return [(int(n), int(F), int(t)) for n, t in zip(Ns, Ts)]


def batch_frame(i: int, inst: Tuple[int, int, int], seed: int = 5,
                T: Optional[int] = None, channels: Optional[Sequence[int]] = None) -> np.ndarray:
    """Samples of batched instance ``i`` (gauss recipe, own stream per instance)."""
    N, F, Tn = inst
    return gen_frame(N, F, Tn if T is None else T, seed, "gauss", channels=channels,
                     stream_key=(_KEY_BATCH, i))
