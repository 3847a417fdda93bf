"""Pins for the CPU oracle: facts fixed by the paper and by the mathematics.

Each ``pin_*`` function takes an oracle library handle and raises
``AssertionError`` when the oracle disagrees with the fact it checks.  The same
functions run against the real oracle (all must pass) and against copies of it
with one planted mistake (at least one must fail), which shows that the pins
would catch that kind of mistake.

None of these re-derive the oracle's own loop: the expected values come from a
hand-worked example, closed forms, invariants of a Gram matrix, numpy complex
arithmetic, or pure-Python complex brute force.
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle
from synth import encode, pack_flags

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _frame(re, im):
    """[T][F][N] bytes from signed parts of the same shape."""
    return encode(np.asarray(re), np.asarray(im))


def _packed_from_full(full_c):
    """int64 [F][B][2] from complex [F][N][N], upper triangle in row-major order."""
    F, N, _ = full_c.shape
    iu, ju = np.triu_indices(N)
    sel = full_c[:, iu, ju]
    return np.stack([sel.real, sel.imag], axis=-1).astype(np.int64)


def _as_complex(re, im):
    return np.asarray(re, dtype=np.float64) + 1j * np.asarray(im, dtype=np.float64)


# ---------------------------------------------------------------- P1 counts
def pin_counts(lib):
    """N(N+1)/2 baselines per channel (Eq. (1); 32,896 at N = 256, Abstract)."""
    for N, nb in ((1, 1), (16, 136), (256, 32896)):
        s = np.full((2, 1, N), 0x88, dtype=np.uint8)
        v = oracle.correlate(s, lib=lib)
        assert v.shape == (1, nb, 2), (N, v.shape)


# ------------------------------------------------------- P2 worked example
def pin_worked_example(lib):
    """Hand-worked two-input example: nibble order, offset, conjugate side, index."""
    with open(os.path.join(GOLDEN, "worked_example.json")) as fh:
        g = json.load(fh)
    for key_s, key_v in (("samples_hex", "vis"), ("nibble_swapped_samples_hex", "nibble_swapped_vis")):
        b = np.array([int(h, 16) for h in g[key_s]], dtype=np.uint8).reshape(g["T"], g["F"], g["N"])
        v = oracle.correlate(b, lib=lib)
        assert v[0].tolist() == g[key_v], (key_s, v[0].tolist())


# ----------------------------------------------------------- P3 closed forms
def pin_extremes(lib):
    """All codes 0x00 (x = -8-8i): V = 128 T; all codes 0x88 (x = 0): V = 0."""
    T, N = 37, 5
    v = oracle.correlate(np.zeros((T, 2, N), np.uint8), lib=lib)
    assert (v[..., 0] == 128 * T).all() and (v[..., 1] == 0).all()
    v = oracle.correlate(np.full((T, 2, N), 0x88, np.uint8), lib=lib)
    assert (v == 0).all()


def pin_constant(lib):
    """Constant inputs c_i: V_ij = T c_i conj(c_j)."""
    rng = np.random.default_rng(11)
    N, T = 7, 19
    cr = rng.integers(-8, 8, N)
    ci = rng.integers(-8, 8, N)
    s = _frame(np.broadcast_to(cr, (T, 1, N)), np.broadcast_to(ci, (T, 1, N)))
    c = _as_complex(cr, ci)
    want = _packed_from_full((T * np.outer(c, c.conj()))[None])
    assert np.array_equal(oracle.correlate(s, lib=lib), want)


def pin_single_tone(lib):
    """x_i(t) = c_i * i^(t + d_i): V_ij = T c_i conj(c_j) i^(d_i - d_j) for T = 0 mod 4.

    Multiplying by i maps Gaussian integers with parts in [-7, 7] onto the same
    set, so the tone stays exactly representable in 4+4 bits.
    """
    rng = np.random.default_rng(12)
    N, T = 6, 64
    c = _as_complex(rng.integers(-7, 8, N), rng.integers(-7, 8, N))
    d = rng.integers(0, 4, N)
    t = np.arange(T)
    x = c[None, :] * (1j ** ((t[:, None] + d[None, :]) % 4))
    x = np.round(x.real) + 1j * np.round(x.imag)
    s = _frame(x.real.astype(int)[:, None, :], x.imag.astype(int)[:, None, :])
    ph = 1j ** ((d[:, None] - d[None, :]) % 4)
    want = _packed_from_full((T * np.outer(c, c.conj()) * ph)[None])
    assert np.array_equal(oracle.correlate(s, lib=lib), want)


def pin_two_tone(lib):
    """x_i(t) = u_i + v_i i^t with T = 0 mod 4: V_ij = T (u_i conj(u_j) + v_i conj(v_j))."""
    rng = np.random.default_rng(13)
    N, T = 5, 40
    u = _as_complex(rng.integers(-3, 4, N), rng.integers(-3, 4, N))
    v = _as_complex(rng.integers(-4, 5, N), rng.integers(-4, 5, N))
    t = np.arange(T)
    x = u[None, :] + v[None, :] * (1j ** (t[:, None] % 4))
    x = np.round(x.real) + 1j * np.round(x.imag)
    s = _frame(x.real.astype(int)[:, None, :], x.imag.astype(int)[:, None, :])
    want = _packed_from_full((T * (np.outer(u, u.conj()) + np.outer(v, v.conj())))[None])
    assert np.array_equal(oracle.correlate(s, lib=lib), want)


# -------------------------------------------------------------- P4 invariants
def _rand_frame(seed, T, F, N, lo=-8, hi=8):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, (T, F, N)), rng.integers(lo, hi, (T, F, N))


def pin_gram_invariants(lib):
    """Hermitian, real non-negative diagonal = sum |x|^2, |V_ij|^2 <= V_ii V_jj."""
    re, im = _rand_frame(21, 50, 2, 9)
    s = _frame(re, im)
    full = oracle.correlate(s, full=True, lib=lib)
    vr, vi = full[..., 0], full[..., 1]
    assert np.array_equal(vr, vr.transpose(0, 2, 1))
    assert np.array_equal(vi, -vi.transpose(0, 2, 1))
    diag_r = np.diagonal(vr, axis1=1, axis2=2)
    assert (np.diagonal(vi, axis1=1, axis2=2) == 0).all()
    p = (re.astype(np.int64) ** 2 + im.astype(np.int64) ** 2).sum(axis=0)  # [F][N]
    assert np.array_equal(diag_r, p)
    mag2 = vr.astype(object) ** 2 + vi.astype(object) ** 2
    dd = diag_r[:, :, None].astype(object) * diag_r[:, None, :].astype(object)
    assert (mag2 <= dd).all()
    # packed triangle agrees with the upper half of the full matrix
    packed = oracle.correlate(s, lib=lib)
    iu, ju = np.triu_indices(9)
    assert np.array_equal(packed, full[:, iu, ju, :])


def pin_time_additivity(lib):
    """V over [0, T) equals V over [0, t) plus V over [t, T)."""
    re, im = _rand_frame(22, 61, 3, 6)
    s = _frame(re, im)
    whole = oracle.correlate(s, lib=lib)
    for cut in (0, 1, 30, 60, 61):
        a = oracle.correlate(s, t0=0, t1=cut, lib=lib)
        b = oracle.correlate(s, t0=cut, t1=61, lib=lib)
        assert np.array_equal(a + b, whole), cut


def pin_symmetries(lib):
    """Input permutation permutes V; nibble swap conjugates V; x -> -x, i x leave V."""
    re, im = _rand_frame(23, 33, 1, 7, lo=-7, hi=8)
    s = _frame(re, im)
    full = oracle.correlate(s, full=True, lib=lib)[0]
    perm = np.random.default_rng(5).permutation(7)
    fp = oracle.correlate(s[:, :, perm], full=True, lib=lib)[0]
    assert np.array_equal(fp, full[perm][:, perm])
    sw = oracle.correlate(_frame(im, re), full=True, lib=lib)[0]
    assert np.array_equal(sw[..., 0], full[..., 0]) and np.array_equal(sw[..., 1], -full[..., 1])
    neg = oracle.correlate(_frame(-re, -im), full=True, lib=lib)[0]
    assert np.array_equal(neg, full)
    rot = oracle.correlate(_frame(-im, re), full=True, lib=lib)[0]
    assert np.array_equal(rot, full)


# ------------------------------------------------- P5 library routine, P6 brute force
def pin_numpy_complex(lib):
    """numpy complex128 X X^H (exact: every partial sum is far below 2^53)."""
    re, im = _rand_frame(31, 300, 3, 33)
    s = _frame(re, im)
    x = _as_complex(re, im)                      # [T][F][N]
    g = np.einsum("tfi,tfj->fij", x, x.conj())   # [F][N][N]
    assert np.array_equal(oracle.correlate(s, lib=lib), _packed_from_full(g))


def pin_brute_force(lib):
    """Pure-Python complex integers on tiny random frames (N <= 4, T <= 4)."""
    rng = np.random.default_rng(41)
    for trial in range(12):
        N = int(rng.integers(1, 5))
        T = int(rng.integers(1, 5))
        F = int(rng.integers(1, 3))
        re = rng.integers(-8, 8, (T, F, N))
        im = rng.integers(-8, 8, (T, F, N))
        got = oracle.correlate(_frame(re, im), lib=lib)
        for f in range(F):
            b = 0
            for i in range(N):
                for j in range(i, N):
                    acc = 0j
                    for t in range(T):
                        xi = complex(int(re[t, f, i]), int(im[t, f, i]))
                        xj = complex(int(re[t, f, j]), int(im[t, f, j]))
                        acc += xi * xj.conjugate()
                    assert got[f, b].tolist() == [int(acc.real), int(acc.imag)], (trial, f, i, j)
                    b += 1


def pin_exhaustive_codes(lib):
    """Every pair of the 256 byte codes, N = 2, T = 1 (each pair as its own channel)."""
    codes = np.arange(256, dtype=np.uint8)
    a, b = np.meshgrid(codes, codes, indexing="ij")
    s = np.stack([a.ravel(), b.ravel()], axis=-1)[None]          # [1][65536][2]
    got = oracle.correlate(s, lib=lib)                            # [65536][3][2]
    # decode by the footnote's definition: stored nibble minus 8, real part high
    val = {c: complex(((c >> 4) & 15) - 8, (c & 15) - 8) for c in range(256)}
    xa = np.array([val[int(c)] for c in a.ravel()])
    xb = np.array([val[int(c)] for c in b.ravel()])
    want = np.stack([xa * xa.conj(), xa * xb.conj(), xb * xb.conj()], axis=1)
    assert np.array_equal(got[..., 0], want.real.astype(np.int64))
    assert np.array_equal(got[..., 1], want.imag.astype(np.int64))


# ------------------------------------------------------------ P7 int32 boundary
def pin_int32_boundary(lib):
    """The largest exact integration: T = 2^24 - 1 of -8-8i gives 2,147,483,520."""
    T = (1 << 24) - 1
    v = oracle.correlate(np.zeros((T, 1, 1), np.uint8), lib=lib)
    assert v[0, 0].tolist() == [2147483520, 0]
    assert 2147483520 <= np.iinfo(np.int32).max < 128 * (1 << 24)


# ------------------------------------------------- time shifting (Sec. IV-C)
def _shift_frame(seed, TT, F, N):
    return np.random.default_rng(seed).integers(0, 256, (TT, F, N), dtype=np.uint8)


def pin_shift_zero_and_uniform(lib):
    """No delay is the plain correlation of the frame; one delay d for every
    input is the plain correlation of the window that starts d rows earlier."""
    D, T, F, N = 9, 40, 2, 7
    ext = _shift_frame(71, D + T, F, N)
    got = oracle.correlate_shifted(ext, D, np.zeros(N, np.int32), lib=lib)
    assert np.array_equal(got, oracle.correlate(ext[D:], lib=lib))
    for d in (1, 5, 9):
        got = oracle.correlate_shifted(ext, D, np.full(N, d, np.int32), lib=lib)
        assert np.array_equal(got, oracle.correlate(ext[D - d:D - d + T], lib=lib)), d


def pin_shift_aligns_delayed_copy(lib):
    """Input 1 carries input 0 late by k samples; delaying input 0 by k lines
    them up, so V_01 becomes the real power of the common signal, and it is
    complex (not aligned) without the delay."""
    D, T, N, k = 12, 64, 3, 5
    ext = _shift_frame(72, D + T, 1, N)
    ext[k:, 0, 1] = ext[:-k, 0, 0]               # x1(r) = x0(r - k)
    delays = np.array([k, 0, 3], np.int32)
    got = oracle.correlate_shifted(ext, D, delays, lib=lib)
    re = (ext[D - k:D - k + T, 0, 0] >> 4).astype(np.int64) - 8
    im = (ext[D - k:D - k + T, 0, 0] & 15).astype(np.int64) - 8
    power = int((re * re + im * im).sum())
    b01 = oracle.tri_index(0, 1, N)
    assert got[0, b01].tolist() == [power, 0]
    assert got[0, oracle.tri_index(0, 0, N)].tolist() == [power, 0]
    plain = oracle.correlate_shifted(ext, D, np.zeros(N, np.int32), lib=lib)
    assert plain[0, b01, 1] != 0


def pin_shift_numpy_complex(lib):
    """Shift the complex samples with numpy indexing and form X X^H (exact)."""
    D, T, F, N = 6, 33, 2, 5
    ext = _shift_frame(73, D + T, F, N)
    delays = np.array([0, 6, 2, 2, 5], np.int32)
    x = _as_complex((ext >> 4).astype(np.int64) - 8, (ext & 15).astype(np.int64) - 8)
    rows = D + np.arange(T)[:, None] - delays[None, :]            # [T][N]
    xs = x[rows, :, np.arange(N)[None, :]]                        # [T][N][F]
    xs = np.transpose(xs, (2, 1, 0))                              # [F][N][T]
    full = np.einsum("fit,fjt->fij", xs, np.conj(xs))
    got = oracle.correlate_shifted(ext, D, delays, lib=lib)
    assert np.array_equal(got, _packed_from_full(np.rint(full.real) + 1j * np.rint(full.imag)))


SHIFT_PINS = (pin_shift_zero_and_uniform, pin_shift_aligns_delayed_copy, pin_shift_numpy_complex)


# ------------------------------------------- flagged data (Sec. IV-A, Data Flow)
def _flag_frame(seed, T, F, N, p):
    rng = np.random.default_rng(seed)
    samples = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    invalid = rng.random((T, F, N)) < p
    return samples, invalid


def pin_flag_none_and_all(lib):
    """No flag gives the plain correlation and T valid pairs everywhere; every
    sample flagged gives zero sums and zero counts, whatever the bytes hold."""
    T, F, N = 37, 2, 35
    samples, _ = _flag_frame(81, T, F, N, 0.0)
    vis, cnt = oracle.correlate_flagged(samples, pack_flags(np.zeros((T, F, N), bool)), lib=lib)
    assert np.array_equal(vis, oracle.correlate(samples, lib=lib))
    assert (cnt == T).all()
    vis, cnt = oracle.correlate_flagged(samples, pack_flags(np.ones((T, F, N), bool)), lib=lib)
    assert not vis.any() and not cnt.any()


def pin_flag_single_input(lib):
    """Input k flagged at a set S of times: every baseline that involves k has
    T - |S| valid pairs, every other one T, and V equals the correlation of
    the frame with k's samples at S set to zero (code 0x88)."""
    T, F, N, k = 50, 1, 6, 3
    samples, _ = _flag_frame(82, T, F, N, 0.0)
    inv = np.zeros((T, F, N), bool)
    S = [0, 7, 8, 9, 31, 49]
    inv[S, 0, k] = True
    vis, cnt = oracle.correlate_flagged(samples, pack_flags(inv), lib=lib)
    for i in range(N):
        for j in range(i, N):
            want = T - len(S) if k in (i, j) else T
            assert cnt[0, oracle.tri_index(i, j, N)] == want, (i, j)
    z = samples.copy()
    z[S, 0, k] = 0x88
    assert np.array_equal(vis, oracle.correlate(z, lib=lib))


def pin_flag_numpy(lib):
    """Counts as the Gram matrix of the validity mask, and V as X X^H of the
    samples multiplied by the mask, both with numpy on random flags."""
    T, F, N = 45, 3, 37
    samples, inv = _flag_frame(83, T, F, N, 0.3)
    valid = (~inv).astype(np.int64)                                  # [T][F][N]
    x = _as_complex((samples >> 4).astype(np.int64) - 8, (samples & 15).astype(np.int64) - 8)
    xm = np.transpose(x * valid, (1, 2, 0))                          # [F][N][T]
    vm = np.transpose(valid, (1, 2, 0))
    full_v = xm @ np.conj(np.transpose(xm, (0, 2, 1)))
    full_c = vm @ np.transpose(vm, (0, 2, 1))
    vis, cnt = oracle.correlate_flagged(samples, pack_flags(inv), lib=lib)
    assert np.array_equal(vis, _packed_from_full(np.rint(full_v.real) + 1j * np.rint(full_v.imag)))
    iu, ju = np.triu_indices(N)
    assert np.array_equal(cnt, full_c[:, iu, ju])


def pin_flag_constant_renormalises(lib):
    """Every valid sample equals c: V_ij = C_ij |c|^2, so renormalising to the
    full integration (scale T) gives exactly T |c|^2 wherever a pair is valid."""
    T, F, N = 64, 2, 9
    c_re, c_im = 3, -5
    samples = encode(np.full((T, F, N), c_re), np.full((T, F, N), c_im))
    _, inv = _flag_frame(84, T, F, N, 0.45)
    inv[:, 1, 4] = True                                              # no valid pair at all
    vis, cnt = oracle.correlate_flagged(samples, pack_flags(inv), lib=lib)
    norm = oracle.normalize(vis, cnt, T)
    p = c_re * c_re + c_im * c_im
    want = np.where(cnt[..., None] > 0, np.array([T * p, 0.0]), 0.0).astype(np.float32)
    assert np.array_equal(norm, want)
    assert (cnt[1, oracle.tri_index(4, 4, N)] == 0) and (cnt < T).any()


# ------------------------------------- discrete beamforming (Sec. IV-C)
def _beam_case(seed, T, F, N, B):
    rng = np.random.default_rng(seed)
    samples = rng.integers(0, 256, (T, F, N), dtype=np.uint8)
    weights = rng.integers(-127, 128, (F, B, N, 2)).astype(np.int8)
    return samples, weights


def _x(samples):
    return _as_complex((samples >> 4).astype(np.int64) - 8, (samples & 15).astype(np.int64) - 8)


def pin_beam_selects_and_rotates(lib):
    """A beam whose only weight is 1 at input k is input k's signal; weight i
    rotates it by 90 degrees (i x = -Im x + i Re x); weight 0 gives 0."""
    T, F, N, B, k = 20, 2, 9, 3, 4
    samples, _ = _beam_case(91, T, F, N, B)
    w = np.zeros((F, B, N, 2), np.int8)
    w[:, 0, k, 0] = 1          # beam 0: x_k
    w[:, 1, k, 1] = 1          # beam 1: i x_k
    y = oracle.beamform(samples, w, lib=lib)
    re = (samples[:, :, k] >> 4).astype(np.int64) - 8
    im = (samples[:, :, k] & 15).astype(np.int64) - 8
    assert np.array_equal(y[:, :, 0, 0], re) and np.array_equal(y[:, :, 0, 1], im)
    assert np.array_equal(y[:, :, 1, 0], -im) and np.array_equal(y[:, :, 1, 1], re)
    assert not y[:, :, 2].any()


def pin_beam_numpy(lib):
    """y = W x per channel and time with numpy complex arithmetic (exact)."""
    T, F, N, B = 17, 3, 21, 5
    samples, w = _beam_case(92, T, F, N, B)
    wc = _as_complex(w[..., 0].astype(np.int64), w[..., 1].astype(np.int64))   # [F][B][N]
    y = np.einsum("fbn,tfn->tfb", wc, _x(samples))
    got = oracle.beamform(samples, w, lib=lib)
    assert np.array_equal(got[..., 0], np.rint(y.real).astype(np.int64))
    assert np.array_equal(got[..., 1], np.rint(y.imag).astype(np.int64))


def pin_beam_power_is_visibility_form(lib):
    """A beam's power summed over time is the quadratic form of the
    correlator's output: sum_t |y_b|^2 = sum_ij w_i conj(w_j) V_ij, with V from
    the oracle's correlation (itself pinned above)."""
    T, F, N, B = 40, 2, 12, 4
    samples, w = _beam_case(93, T, F, N, B)
    y = oracle.beamform(samples, w, lib=lib)
    power = (y[..., 0] ** 2 + y[..., 1] ** 2).sum(axis=0)                         # [F][B]
    V = oracle.correlate(samples, full=True, lib=lib)                             # [F][N][N][2]
    Vc = V[..., 0] + 1j * V[..., 1]
    wc = w[..., 0].astype(np.float64) + 1j * w[..., 1].astype(np.float64)
    q = np.einsum("fbi,fij,fbj->fb", wc, Vc, np.conj(wc))
    assert np.array_equal(power, np.rint(q.real).astype(np.int64))
    assert np.allclose(q.imag, 0)


BEAM_PINS = (pin_beam_selects_and_rotates, pin_beam_numpy, pin_beam_power_is_visibility_form)


FLAG_PINS = (pin_flag_none_and_all, pin_flag_single_input, pin_flag_numpy,
             pin_flag_constant_renormalises)

FAST_PINS = (pin_counts, pin_worked_example, pin_extremes, pin_constant, pin_single_tone,
             pin_two_tone, pin_gram_invariants, pin_time_additivity, pin_symmetries,
             pin_numpy_complex, pin_brute_force, pin_exhaustive_codes)
ALL_PINS = FAST_PINS + (pin_int32_boundary,)
