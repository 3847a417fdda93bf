/*
 * CPU oracle for the correlator X-engine -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path never calls it and shares no code,
 * header or table with it.
 *
 * What it computes is the plain definition of the X-engine's output (Sec. I and
 * Sec. IV-C, "Full Correlation"): for every frequency channel f, the integrated
 * pairwise products of all inputs,
 *
 *     V_f[i][j] = sum over t of x[t][f][i] * conj(x[t][f][j]),   0 <= i <= j < N,
 *
 * i.e. the N(N+1)/2 baselines of Eq. (1), autocorrelations included.  Each
 * sample is one byte: real part in the high nibble, imaginary part in the low
 * nibble, both offset-binary (stored = value + 8, Sec. II-A footnote).
 *
 * Readings where the paper is silent: the conjugate goes on the second input
 * (x_i * conj(x_j)); baselines are stored row-major over the upper triangle,
 * b(i, j) = i*N - i*(i-1)/2 + (j - i); each baseline is an interleaved (re, im)
 * pair.  Sums are kept in int64 so that the oracle itself cannot overflow.
 *
 * Loop order is the definition's: channel, row, column, time.  The only step
 * before the loops is decoding one channel's bytes into signed parts.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* The offset of the 4-bit offset-binary code (Sec. II-A footnote). */
#ifdef ORACLE_MUTANT_OFFSET
#define ORACLE_OFFSET 7                 /* planted mistake: wrong offset */
#else
#define ORACLE_OFFSET 8
#endif

/* Offset-binary nibble to signed value. */
static inline int nib_real(uint8_t b) {
#ifdef ORACLE_MUTANT_NIBBLE
    return (int)(b & 15u) - ORACLE_OFFSET;   /* planted mistake: nibbles swapped */
#else
    return (int)(b >> 4) - ORACLE_OFFSET;
#endif
}

static inline int nib_imag(uint8_t b) {
#ifdef ORACLE_MUTANT_NIBBLE
    return (int)(b >> 4) - ORACLE_OFFSET;
#else
    return (int)(b & 15u) - ORACLE_OFFSET;
#endif
}

/* Packed upper-triangle index of baseline (i, j), i <= j. */
static inline int64_t tri_index(int64_t i, int64_t j, int64_t N) {
#ifdef ORACLE_MUTANT_INDEX
    return j * (j + 1) / 2 + i;         /* planted mistake: column-major triangle */
#else
    return i * N - i * (i - 1) / 2 + (j - i);
#endif
}

int oracle_version(void) { return 1; }

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * samples: host [T][F][N] bytes.  channels: F_sel channel indices to correlate
 * (NULL means all F, in order).  out: host int64, [F_sel][N(N+1)/2][2] when
 * full == 0, or the whole Hermitian matrix [F_sel][N][N][2] when full != 0.
 * t0, t1: the time range [t0, t1) to integrate.
 * Returns 0, or -1 on bad arguments, -2 when memory runs out.
 */
int oracle_correlate_range(const uint8_t *samples, int N, int F, int T,
                           const int *channels, int F_sel, int t0, int t1,
                           int64_t *out, int full) {
    if (!samples || !out || N < 1 || F < 1 || T < 0 || F_sel < 0 ||
        t0 < 0 || t1 < t0 || t1 > T)
        return -1;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    const int64_t per_chan = full ? (int64_t)N * N * 2 : nb * 2;
    const int64_t Tn = (int64_t)t1 - t0;
    signed char *re = (signed char *)malloc((size_t)(N * Tn > 0 ? N * Tn : 1));
    signed char *im = (signed char *)malloc((size_t)(N * Tn > 0 ? N * Tn : 1));
    if (!re || !im) {
        free(re);
        free(im);
        return -2;
    }
    for (int k = 0; k < F_sel; ++k) {
        const int f = channels ? channels[k] : k;
        if (f < 0 || f >= F) {
            free(re);
            free(im);
            return -1;
        }
        /* decode this channel: re[n][t], im[n][t] */
        for (int64_t t = 0; t < Tn; ++t) {
            const uint8_t *row = samples + ((t0 + t) * (int64_t)F + f) * N;
            for (int n = 0; n < N; ++n) {
                re[n * Tn + t] = (signed char)nib_real(row[n]);
                im[n * Tn + t] = (signed char)nib_imag(row[n]);
            }
        }
        int64_t *o = out + (int64_t)k * per_chan;
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < N; ++i) {
            const signed char *ri = re + (int64_t)i * Tn, *mi = im + (int64_t)i * Tn;
            for (int j = full ? 0 : i; j < N; ++j) {
                const signed char *rj = re + (int64_t)j * Tn, *mj = im + (int64_t)j * Tn;
                int64_t acc_re = 0, acc_im = 0;
#ifdef ORACLE_MUTANT_TLAST
                for (int64_t t = 0; t + 1 < Tn; ++t) {   /* planted mistake: last sample dropped */
#else
                for (int64_t t = 0; t < Tn; ++t) {
#endif
                    /* (a + ib)(c - id) = (ac + bd) + i(bc - ad) */
#ifdef ORACLE_MUTANT_DROP
                    acc_re += (int64_t)ri[t] * rj[t];          /* planted mistake: dropped term */
#else
                    acc_re += (int64_t)ri[t] * rj[t] + (int64_t)mi[t] * mj[t];
#endif
#ifdef ORACLE_MUTANT_CONJ
                    acc_im += (int64_t)ri[t] * mj[t] - (int64_t)mi[t] * rj[t];
#else
                    acc_im += (int64_t)mi[t] * rj[t] - (int64_t)ri[t] * mj[t];
#endif
                }
                const int64_t b = full ? (int64_t)i * N + j : tri_index(i, j, N);
                o[2 * b] = acc_re;
                o[2 * b + 1] = acc_im;
            }
        }
    }
    free(re);
    free(im);
    return 0;
}

/* All channels, the whole integration [0, T). */
int oracle_correlate(const uint8_t *samples, int N, int F, int T, int64_t *out, int full) {
    return oracle_correlate_range(samples, N, F, T, NULL, F, 0, T, out, full);
}

/*
 * Output gating (Sec. IV-C, "Output Gating"): the integration is split into G
 * sub-buffers by a per-sample gate index; a sample with gate[t] outside [0, G)
 * goes to no buffer.  out: [G][F][N(N+1)/2][2] int64.  This is the same
 * definition as above with the time sum restricted to {t : gate[t] == g}.
 */
int oracle_correlate_gated(const uint8_t *samples, int N, int F, int T,
                           const int *gate, int G, int64_t *out) {
    if (!samples || !gate || !out || N < 1 || F < 1 || T < 0 || G < 1)
        return -1;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    memset(out, 0, sizeof(int64_t) * (size_t)(G * F * nb * 2));
    for (int f = 0; f < F; ++f) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < N; ++i) {
            for (int j = i; j < N; ++j) {
                const int64_t b = tri_index(i, j, N);
                for (int t = 0; t < T; ++t) {
                    const int g = gate[t];
                    if (g < 0 || g >= G) continue;
                    const uint8_t si = samples[((int64_t)t * F + f) * N + i];
                    const uint8_t sj = samples[((int64_t)t * F + f) * N + j];
                    const int64_t a = nib_real(si), bi = nib_imag(si);
                    const int64_t c = nib_real(sj), d = nib_imag(sj);
                    int64_t *o = out + (((int64_t)g * F + f) * nb + b) * 2;
                    o[0] += a * c + bi * d;
                    o[1] += bi * c - a * d;
                }
            }
        }
    }
    return 0;
}

/*
 * Time shifting (Sec. IV-C, "Time Shifting"): input i is delayed by delays[i]
 * samples before it is correlated, x'_i(t) = x_i(t - delays[i]).  `ext` holds
 * D_max samples of history followed by the T samples of the frame,
 * [D_max + T][F][N], so frame time t is row D_max + t and a delayed sample
 * reaches back at most D_max rows.  out: [F][N(N+1)/2][2] as above.
 */
int oracle_correlate_shifted(const uint8_t *ext, int N, int F, int T, int D_max,
                             const int *delays, int64_t *out) {
    if (!ext || !delays || !out || N < 1 || F < 1 || T < 0 || D_max < 0) return -1;
    for (int i = 0; i < N; ++i)
        if (delays[i] < 0 || delays[i] > D_max) return -1;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    memset(out, 0, sizeof(int64_t) * (size_t)(F * nb * 2));
    for (int f = 0; f < F; ++f) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < N; ++i) {
            for (int j = i; j < N; ++j) {
                int64_t re = 0, im = 0;
                for (int t = 0; t < T; ++t) {
#ifdef ORACLE_MUTANT_SHIFT
                    /* planted mistake: the delay applied to the other input */
                    const uint8_t si = ext[((int64_t)(D_max + t - delays[j]) * F + f) * N + i];
                    const uint8_t sj = ext[((int64_t)(D_max + t - delays[i]) * F + f) * N + j];
#else
                    const uint8_t si = ext[((int64_t)(D_max + t - delays[i]) * F + f) * N + i];
                    const uint8_t sj = ext[((int64_t)(D_max + t - delays[j]) * F + f) * N + j];
#endif
                    const int64_t a = nib_real(si), bi = nib_imag(si);
                    const int64_t c = nib_real(sj), d = nib_imag(sj);
                    re += a * c + bi * d;
                    im += bi * c - a * d;
                }
                int64_t *o = out + ((int64_t)f * nb + tri_index(i, j, N)) * 2;
                o[0] = re;
                o[1] = im;
            }
        }
    }
    return 0;
}

/*
 * Flagged data (Sec. IV-A, "Data Flow"): lost packets and F-engine flags
 * (ADC saturation, FFT overflow) mark samples as invalid, and the count of
 * such data renormalises the integrated matrices.  A flagged sample takes no
 * part in the integration, whatever its byte holds:
 *
 *     V_f[i][j] = sum over t with both samples valid of x_i conj(x_j),
 *     C_f[i][j] = number of t with both x[t][f][i] and x[t][f][j] valid.
 *
 * flags: uint32 [T][F][W], W = ceil(N / 32); bit (i % 32) of word i / 32 set
 * means sample (t, f, i) is invalid.  out: [F][N(N+1)/2][2] as above;
 * counts: int64 [F][N(N+1)/2].
 */
static inline int flagged(const uint32_t *flags, int64_t t, int f, int i, int F, int W) {
    return (int)((flags[(t * F + f) * W + (i >> 5)] >> (i & 31)) & 1u);
}

int oracle_correlate_flagged(const uint8_t *samples, const uint32_t *flags, int N, int F, int T,
                             int64_t *out, int64_t *counts) {
    if (!samples || !flags || !out || !counts || N < 1 || F < 1 || T < 0) return -1;
    const int W = (N + 31) / 32;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    for (int f = 0; f < F; ++f) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < N; ++i) {
            for (int j = i; j < N; ++j) {
                int64_t re = 0, im = 0, n = 0;
                for (int t = 0; t < T; ++t) {
#ifdef ORACLE_MUTANT_FLAG
                    /* planted mistake: only the first input's flag is honoured */
                    if (flagged(flags, t, f, i, F, W)) continue;
#else
                    if (flagged(flags, t, f, i, F, W) || flagged(flags, t, f, j, F, W)) continue;
#endif
                    const uint8_t si = samples[((int64_t)t * F + f) * N + i];
                    const uint8_t sj = samples[((int64_t)t * F + f) * N + j];
                    const int64_t a = nib_real(si), bi = nib_imag(si);
                    const int64_t c = nib_real(sj), d = nib_imag(sj);
                    re += a * c + bi * d;
                    im += bi * c - a * d;
                    ++n;
                }
                const int64_t b = (int64_t)f * nb + tri_index(i, j, N);
                out[b * 2] = re;
                out[b * 2 + 1] = im;
                counts[b] = n;
            }
        }
    }
    return 0;
}

/*
 * Discrete beamforming (Sec. IV-C, "Discrete Beamforming"): the data of all
 * inputs are phase-shifted and summed, so that signals from one direction add
 * in phase; the summed signal is written out at the sample cadence.  For every
 * time t, channel f and beam b,
 *
 *     y[t][f][b] = sum over n of w[f][b][n] * x[t][f][n]
 *
 * with complex integer weights (the phases, scaled and rounded by the caller)
 * applied as given, without a conjugate.  weights: int8 [F][B][N][2] (re, im);
 * out: int64 [T][F][B][2] (re, im).
 */
int oracle_beamform(const uint8_t *samples, const int8_t *weights, int N, int F, int T, int B,
                    int64_t *out) {
    if (!samples || !weights || !out || N < 1 || F < 1 || T < 0 || B < 1) return -1;
#pragma omp parallel for schedule(static)
    for (int t = 0; t < T; ++t) {
        for (int f = 0; f < F; ++f) {
            const uint8_t *x = samples + ((int64_t)t * F + f) * N;
            for (int b = 0; b < B; ++b) {
                const int8_t *w = weights + (((int64_t)f * B + b) * N) * 2;
                int64_t re = 0, im = 0;
                for (int n = 0; n < N; ++n) {
                    const int64_t xr = nib_real(x[n]), xi = nib_imag(x[n]);
#ifdef ORACLE_MUTANT_BEAMCONJ
                    const int64_t wr = w[2 * n], wi = -w[2 * n + 1];   /* planted mistake: conj(w) */
#else
                    const int64_t wr = w[2 * n], wi = w[2 * n + 1];
#endif
                    re += wr * xr - wi * xi;
                    im += wr * xi + wi * xr;
                }
                int64_t *o = out + (((int64_t)t * F + f) * B + b) * 2;
                o[0] = re;
                o[1] = im;
            }
        }
    }
    return 0;
}

/*
 * Selected baselines only: out[k] = V_{f[k]}[i[k]][j[k]] as (re, im), summed
 * over t in [0, T) straight from the sample bytes (the same definition as
 * above, one baseline at a time), for checking full-size frames at sampled
 * outputs.  Any i, j order is accepted (i > j gives the conjugate).
 */
int oracle_correlate_pairs(const uint8_t *samples, int N, int F, int T, const int *fs,
                           const int *is, const int *js, int npairs, int64_t *out) {
    if (!samples || !fs || !is || !js || !out || N < 1 || F < 1 || T < 0 || npairs < 0)
        return -1;
    for (int k = 0; k < npairs; ++k)
        if (fs[k] < 0 || fs[k] >= F || is[k] < 0 || is[k] >= N || js[k] < 0 || js[k] >= N)
            return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < npairs; ++k) {
        const int64_t f = fs[k], i = is[k], j = js[k];
        int64_t acc_re = 0, acc_im = 0;
        for (int64_t t = 0; t < T; ++t) {
            const uint8_t si = samples[(t * F + f) * N + i];
            const uint8_t sj = samples[(t * F + f) * N + j];
            const int64_t a = nib_real(si), b = nib_imag(si);
            const int64_t c = nib_real(sj), d = nib_imag(sj);
            acc_re += a * c + b * d;
            acc_im += b * c - a * d;
        }
        out[2 * k] = acc_re;
        out[2 * k + 1] = acc_im;
    }
    return 0;
}
