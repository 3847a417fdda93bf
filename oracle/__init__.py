"""CPU oracle of the X-engine correlation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP path.

``correlate`` returns the plain definition of the X-engine output (Sec. I;
Sec. IV-C, "Full Correlation"; Eq. (1) counts the N(N+1)/2 baselines):
``V_f[i][j] = sum_t x_i conj(x_j)`` over the upper triangle including the
diagonal, as int64 ``[F][N(N+1)/2][2]`` (re, im), computed by the C loop nest in
``xeng_oracle.c``.

Parity pins (see ``tests/test_oracle_pins.py``): a hand-worked example, closed
forms for constant, single-tone and two-tone inputs, Gram-matrix invariants,
numpy complex128 ``X @ X^H``, pure-Python brute force, the exhaustive 256 x 256
code pairs and the int32 boundary.  The gated variant is pinned by summing its
gates back to the ungated result and by brute force; the shifted and flagged
variants and the beamformer have pins of their own.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_LIBS: dict = {}


def load(mutant: Optional[str] = None, path: Optional[str] = None) -> ctypes.CDLL:
    """Load (building it first if absent) the oracle library."""
    if not path and not mutant and os.environ.get("ORACLE_LIBRARY"):
        path = os.environ["ORACLE_LIBRARY"]  # another build of the same source
    key = path or mutant or ""
    if key in _LIBS:
        return _LIBS[key]
    p = path or _build.lib_path(mutant)
    if not os.path.exists(p):
        p = _build.build(mutant)
    lib = ctypes.CDLL(p)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_correlate_range.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p,
                                           ctypes.c_int]
    lib.oracle_correlate_range.restype = ctypes.c_int
    lib.oracle_correlate_gated.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip,
                                           ctypes.c_int, i64p]
    lib.oracle_correlate_gated.restype = ctypes.c_int
    lib.oracle_correlate_pairs.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, ip,
                                           ctypes.c_int, i64p]
    lib.oracle_correlate_pairs.restype = ctypes.c_int
    lib.oracle_correlate_shifted.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ip, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_correlate_shifted.restype = ctypes.c_int
    lib.oracle_correlate_flagged.argtypes = [u8p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, i64p, i64p]
    lib.oracle_correlate_flagged.restype = ctypes.c_int
    lib.oracle_beamform.argtypes = [u8p, ctypes.POINTER(ctypes.c_int8), ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, i64p]
    lib.oracle_beamform.restype = ctypes.c_int
    lib.oracle_threads.restype = ctypes.c_int
    _LIBS[key] = lib
    return lib


def threads(lib: Optional[ctypes.CDLL] = None) -> int:
    return int((lib or load()).oracle_threads())


def correlate(samples: np.ndarray, channels: Optional[Sequence[int]] = None,
              t0: int = 0, t1: Optional[int] = None, full: bool = False,
              lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """Visibilities of ``samples[T][F][N]`` (uint8).

    Returns int64 ``[F_sel][N(N+1)/2][2]``, or ``[F_sel][N][N][2]`` (the whole
    Hermitian matrix) with ``full=True``; ``channels`` selects channels and
    ``[t0, t1)`` the integrated time range.
    """
    s = np.ascontiguousarray(samples, dtype=np.uint8)
    if s.ndim != 3:
        raise ValueError("samples must be [T][F][N]")
    T, F, N = s.shape
    t1 = T if t1 is None else int(t1)
    chans = list(range(F)) if channels is None else [int(c) for c in channels]
    nb = N * (N + 1) // 2
    shape = (len(chans), N, N, 2) if full else (len(chans), nb, 2)
    out = np.zeros(shape, dtype=np.int64)
    ch = (ctypes.c_int * max(1, len(chans)))(*chans)
    lib = lib or load()
    rc = lib.oracle_correlate_range(
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), N, F, T, ch, len(chans), int(t0), t1,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1 if full else 0)
    if rc != 0:
        raise ValueError(f"oracle_correlate_range failed ({rc})")
    return out


def correlate_gated(samples: np.ndarray, gate: np.ndarray, G: int,
                    lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """Gated visibilities int64 ``[G][F][N(N+1)/2][2]``; ``gate[t]`` picks the buffer."""
    s = np.ascontiguousarray(samples, dtype=np.uint8)
    T, F, N = s.shape
    g = np.ascontiguousarray(gate, dtype=np.int32)
    if g.shape != (T,):
        raise ValueError("gate must have one entry per time sample")
    nb = N * (N + 1) // 2
    out = np.zeros((G, F, nb, 2), dtype=np.int64)
    lib = lib or load()
    rc = lib.oracle_correlate_gated(
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), N, F, T,
        g.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(G),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_correlate_gated failed ({rc})")
    return out


def correlate_shifted(ext: np.ndarray, D_max: int, delays: np.ndarray,
                      lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """Visibilities int64 [F][N(N+1)/2][2] of inputs delayed by ``delays`` samples.

    ``ext`` is [D_max + T][F][N]: D_max samples of history, then the frame.
    """
    e = np.ascontiguousarray(ext, dtype=np.uint8)
    TT, F, N = e.shape
    T = TT - int(D_max)
    d = np.ascontiguousarray(delays, dtype=np.int32)
    if T < 0 or d.shape != (N,):
        raise ValueError("ext must hold D_max + T rows and delays one entry per input")
    out = np.zeros((F, N * (N + 1) // 2, 2), dtype=np.int64)
    lib = lib or load()
    rc = lib.oracle_correlate_shifted(e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), N, F, T,
                                      int(D_max), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_correlate_shifted failed ({rc})")
    return out


def correlate_flagged(samples: np.ndarray, flags: np.ndarray,
                      lib: Optional[ctypes.CDLL] = None):
    """Visibilities and valid-pair counts of a frame with invalid samples.

    ``flags`` is uint32 ``[T][F][ceil(N/32)]``, bit ``i % 32`` of word ``i // 32``
    set when sample ``(t, f, i)`` is invalid.  Returns ``(vis, counts)``: int64
    ``[F][N(N+1)/2][2]`` summed over the times where both inputs are valid, and
    int64 ``[F][N(N+1)/2]``, the number of such times.
    """
    s = np.ascontiguousarray(samples, dtype=np.uint8)
    T, F, N = s.shape
    fl = np.ascontiguousarray(flags, dtype=np.uint32)
    if fl.shape != (T, F, (N + 31) // 32):
        raise ValueError("flags must be uint32 [T][F][ceil(N/32)]")
    nb = N * (N + 1) // 2
    out = np.zeros((F, nb, 2), dtype=np.int64)
    counts = np.zeros((F, nb), dtype=np.int64)
    lib = lib or load()
    rc = lib.oracle_correlate_flagged(
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
        fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), N, F, T,
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_correlate_flagged failed ({rc})")
    return out, counts


def normalize(vis: np.ndarray, counts: np.ndarray, scale: float) -> np.ndarray:
    """Renormalised visibilities, float32 ``[F][N(N+1)/2][2]``.

    Each baseline's integrated sum is rescaled by the fraction of valid pairs:
    ``V * scale / C`` in float64, rounded once to float32, and 0 where C == 0
    (no valid pair).  With ``scale`` = the number of samples integrated this is
    the sum the integration would have had with no data missing; with
    ``scale`` = 1 it is the mean product per valid sample.
    """
    v = np.asarray(vis, dtype=np.float64)
    c = np.asarray(counts, dtype=np.float64)[..., None]
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(c > 0, v * float(scale) / c, 0.0)
    return out.astype(np.float32)


def beamform(samples: np.ndarray, weights: np.ndarray,
             lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """Beams int64 ``[T][F][B][2]``: ``y = sum_n w[f][b][n] x[t][f][n]``.

    ``weights`` is int8 ``[F][B][N][2]`` (re, im), applied without a conjugate.
    """
    s = np.ascontiguousarray(samples, dtype=np.uint8)
    T, F, N = s.shape
    w = np.ascontiguousarray(weights, dtype=np.int8)
    if w.ndim != 4 or w.shape[0] != F or w.shape[2] != N or w.shape[3] != 2:
        raise ValueError("weights must be int8 [F][B][N][2]")
    B = w.shape[1]
    out = np.zeros((T, F, B, 2), dtype=np.int64)
    lib = lib or load()
    rc = lib.oracle_beamform(s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                             w.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), N, F, T, B,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_beamform failed ({rc})")
    return out


def correlate_pairs(samples: np.ndarray, f: np.ndarray, i: np.ndarray, j: np.ndarray,
                    lib: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """V_f[i][j] (int64 re, im) for selected baselines, one by one."""
    s = np.ascontiguousarray(samples, dtype=np.uint8)
    T, F, N = s.shape
    fa, ia, ja = (np.ascontiguousarray(x, dtype=np.int32) for x in (f, i, j))
    if not (fa.shape == ia.shape == ja.shape) or fa.ndim != 1:
        raise ValueError("f, i, j must be equal-length 1-D arrays")
    out = np.zeros((len(fa), 2), dtype=np.int64)
    ip = ctypes.POINTER(ctypes.c_int)
    lib = lib or load()
    rc = lib.oracle_correlate_pairs(
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), N, F, T, fa.ctypes.data_as(ip),
        ia.ctypes.data_as(ip), ja.ctypes.data_as(ip), len(fa),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_correlate_pairs failed ({rc})")
    return out


def tri_index(i: int, j: int, N: int) -> int:
    """Row-major upper-triangle position of baseline (i, j), i <= j."""
    return i * N - i * (i - 1) // 2 + (j - i)


def to_int32(v: np.ndarray) -> np.ndarray:
    """Narrow oracle sums to the int32 output type, refusing any that do not fit."""
    if v.size and (v.min() < np.iinfo(np.int32).min or v.max() > np.iinfo(np.int32).max):
        raise OverflowError("visibility outside int32")
    return v.astype(np.int32)
