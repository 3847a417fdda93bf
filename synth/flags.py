"""Seeded synthetic flag masks: which samples of a frame are invalid.

The F-engine sends flags with its data (Sec. IV-A, "Data Flow"): packets lost
on the way to the GPU nodes, ADC saturation and FFT channelizer overflow.  A
flag mask is packed as uint32 ``[T][F][ceil(N/32)]``; bit ``i % 32`` of word
``i // 32`` is set when sample ``(t, f, i)`` is invalid.  Bits for inputs
``i >= N`` in the last word mean nothing and may be set.

Recipe ``pathfinder`` (all draws from numpy PCG64 seeded through
``SeedSequence``), built directly in packed form so that full-size masks stay
small:

* packet loss: time is cut into packets of ``packet_len`` samples and channels
  into links of ``link_channels``; each (packet, link) is lost with probability
  ``p_packet``, and then every input of those samples is invalid (one link
  carries all inputs of a set of channels);
* ADC saturation: each (input, block of ``sat_len`` samples) saturates with
  probability ``p_sat``; that input is then invalid in every channel for the
  block (saturation precedes the channelizer);
* FFT overflow: single samples ``(t, f, i)`` with probability ``p_fft``.

The defaults (1e-3, 1e-3, 1e-5) model a healthy array with rare faults;
``heavy`` raises packet loss to 5% and saturation to 2%, so that most times
have several inputs invalid.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

_KEY_FLAGS = 0xF1A


def words(N: int) -> int:
    return (N + 31) // 32


def pack_flags(invalid: np.ndarray) -> np.ndarray:
    """Pack a boolean ``[T][F][N]`` mask (True = invalid) into uint32 words."""
    m = np.asarray(invalid, dtype=bool)
    T, F, N = m.shape
    W = words(N)
    pad = np.zeros((T, F, W * 32), dtype=bool)
    pad[:, :, :N] = m
    by = np.packbits(pad, axis=-1, bitorder="little")           # [T][F][4W] bytes
    return np.ascontiguousarray(by).view("<u4").reshape(T, F, W).astype(np.uint32)


def unpack_flags(flags: np.ndarray, N: int) -> np.ndarray:
    """Boolean ``[T][F][N]`` from packed words (bits beyond N dropped)."""
    fl = np.ascontiguousarray(flags, dtype="<u4")
    T, F, W = fl.shape
    bits = np.unpackbits(fl.view(np.uint8).reshape(T, F, 4 * W), axis=-1, bitorder="little")
    return bits[:, :, :N].astype(bool)


def gen_flags(T: int, F: int, N: int, seed: int, recipe: str = "pathfinder",
              packet_len: int = 16, link_channels: int = 8, sat_len: int = 64,
              p_packet: Optional[float] = None, p_sat: Optional[float] = None,
              p_fft: Optional[float] = None) -> np.ndarray:
    """A packed flag mask uint32 ``[T][F][ceil(N/32)]`` (see the module text)."""
    base = {"pathfinder": (1e-3, 1e-3, 1e-5), "heavy": (5e-2, 2e-2, 1e-4),
            "none": (0.0, 0.0, 0.0)}
    if recipe not in base:
        raise ValueError(f"unknown flag recipe {recipe!r}")
    dp, ds, df = base[recipe]
    p_packet = dp if p_packet is None else p_packet
    p_sat = ds if p_sat is None else p_sat
    p_fft = df if p_fft is None else p_fft
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, _KEY_FLAGS])))
    W = words(N)
    fl = np.zeros((T, F, W), dtype=np.uint32)
    full = np.full(W, 0xFFFFFFFF, dtype=np.uint32)
    if N % 32:
        full[-1] = np.uint32((1 << (N % 32)) - 1)
    # packet loss: (packet, link) pairs
    npk, nlk = -(-T // packet_len), -(-F // link_channels)
    lost = np.argwhere(rng.random((npk, nlk)) < p_packet)
    for pk, lk in lost:
        fl[pk * packet_len:(pk + 1) * packet_len, lk * link_channels:(lk + 1) * link_channels] |= full
    # ADC saturation: (input, block) pairs, all channels
    nsb = -(-T // sat_len)
    sat = np.argwhere(rng.random((N, nsb)) < p_sat)
    for i, sb in sat:
        fl[sb * sat_len:(sb + 1) * sat_len, :, i >> 5] |= np.uint32(1 << (i & 31))
    # FFT overflow: single samples
    n = int(rng.binomial(T * F * N, p_fft)) if p_fft > 0 else 0
    if n:
        t = rng.integers(0, T, n)
        f = rng.integers(0, F, n)
        i = rng.integers(0, N, n)
        np.bitwise_or.at(fl, (t, f, i >> 5), (np.uint32(1) << (i & 31).astype(np.uint32)))
    return fl
