/*
 * xeng.h -- C ABI of the MI355X (gfx950) correlator X-engine.
 *
 * The engine computes, for every frequency channel f of a frame of 4+4-bit
 * complex samples, the integrated pairwise products of all inputs (Sec. I;
 * Sec. IV-C, "Full Correlation"):
 *
 *     V_f[i][j] = sum_{t < T} x[t][f][i] * conj(x[t][f][j]),   0 <= i <= j < N,
 *
 * the N(N+1)/2 baselines of Eq. (1), autocorrelations included.  All sums are
 * exact integers.
 *
 * Data layout (shared by every entry point):
 *   samples  device memory, uint8 [T][F][N] (N fastest).  One byte per complex
 *            sample: high nibble = real part + 8, low nibble = imaginary part
 *            + 8 (offset binary, Sec. II-A footnote).  Every byte is a valid
 *            sample; there is no reserved code.
 *   vis      device memory, int32 [F][N(N+1)/2][2]: for each channel the upper
 *            triangle in row-major order, baseline (i, j) at
 *            b(i, j) = i*N - i*(i-1)/2 + (j - i), stored as (re, im).
 *            Im of every autocorrelation (i == j) is 0.
 *
 * Ownership: samples and vis belong to the caller; the library neither frees
 * them nor keeps them past the call.  A plan owns its own workspace.
 *
 * Execution: every compute entry point is asynchronous and ordered on the
 * caller's HIP stream (a hipStream_t passed as void*; NULL is the null
 * stream).  No host synchronisation and no host allocation happen on the call
 * path of xeng_correlate.  A plan is not re-entrant: at most one call in flight
 * per plan; distinct plans are independent.
 *
 * Errors: functions return XENG_OK (0) or a negative code; nothing throws
 * across the ABI.  XENG_EINVAL, XENG_EPLAN and XENG_EOVERFLOW are decided on
 * the host before any HIP call, so they are reported even without a GPU.
 * XENG_EHIP carries a HIP runtime or launch error; its text is kept per plan
 * (xeng_plan_error).
 *
 * Exactness: int32 holds every result while T <= 2^24 - 1 (|Re| <= 128 T).
 * Calls with a larger T fail with XENG_EOVERFLOW; integrate longer by calling
 * again with XENG_ACCUMULATE and dumping before int32 would overflow.
 */
#ifndef XENG_H
#define XENG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xeng_plan_s *xeng_plan_t;

enum {
    XENG_OK = 0,
    XENG_EINVAL = -1,    /* bad argument: size < 1, NULL pointer, unknown flag */
    XENG_EPLAN = -2,     /* argument disagrees with the plan (N, F, T > T_max, count) */
    XENG_EOVERFLOW = -3, /* T > XENG_T_EXACT_MAX: int32 could overflow */
    XENG_EHIP = -4,      /* HIP runtime or launch error (text: xeng_plan_error) */
    XENG_ENOMEM = -5,    /* host or device workspace allocation failed */
    XENG_ELIMIT = -6     /* request exceeds the fixed workspace of xeng_correlate_batch_noalloc */
};

/* Flags of xeng_plan / xeng_plan_batch. */
enum {
    XENG_FORM_I8 = 0,        /* int8 MFMA, int32 accumulators (default) */
    XENG_FORM_F8 = 1,        /* FP8 e4m3 MFMA, f32 accumulators flushed to int32 */
    XENG_FORM_MASK = 0xff,
    XENG_ACCUMULATE = 1 << 8, /* add into vis instead of overwriting it */
    XENG_SHARED_VIS = 1 << 9  /* batch plans only, with XENG_ACCUMULATE: instances may share
                                 a vis buffer; every write is an int32 atomic add (exact) */
};

#define XENG_T_EXACT_MAX 16777215 /* 2^24 - 1 */
#define XENG_N_MAX 32768          /* inputs per instance, at most */
#define XENG_F8_FLUSH_MAX 32768   /* FP8 form: samples per f32 partial sum, at most (sums of
                                     codes 0..15 stay below 2 * 225 * 32768 < 2^24) */
#define XENG_G_MAX 65536          /* output gating: gate buffers per plan, at most */
#define XENG_BEAMS_MAX 1024       /* beams per beamforming plan, at most */
#define XENG_I8_SEG_MAX 524288    /* int8 form, 128 x 128 tiles: samples integrated per launch
                                     (or per batch slice), at most; the int32 sums of codes
                                     then stay below 2^31.  Longer frames are split into
                                     launches that add in stream order (or into more slices). */
#define XENG_NOALLOC_INST_MAX 64      /* xeng_correlate_batch_noalloc: active instances per call */
#define XENG_NOALLOC_ITEMS_MAX 65536  /* xeng_correlate_batch_noalloc: work items per call */

/* Library version: (major << 16) | minor. */
int xeng_version(void);

/* Text of an error code (static storage). */
const char *xeng_strerror(int code);

/*
 * Create a plan for frames of N inputs, F channels and at most T_max samples
 * (the X-engine of Sec. IV-C, "Full Correlation": one frequency band per
 * channel, N(N+1)/2 baselines each by Eq. (1)).
 * flags: one XENG_FORM_* value, optionally | XENG_ACCUMULATE.  The plan does
 * no HIP call; workspace, if a call needs any, is allocated on first use.
 * Errors: XENG_EINVAL (out NULL, N, F or T_max < 1, N > XENG_N_MAX, unknown flag bits),
 * XENG_EOVERFLOW (T_max > XENG_T_EXACT_MAX), XENG_ENOMEM.
 */
int xeng_plan(xeng_plan_t *out, int N, int F, int T_max, unsigned flags);

/*
 * Correlate one frame: vis (see layout above) from samples[T][F][N], the
 * integrated pairwise products of all inputs in every band (Sec. I; Sec. IV-C,
 * "Full Correlation"; Eq. (1)) on the offset-binary samples of Sec. II-A.
 * N and F must equal the plan's, 1 <= T <= T_max.  With XENG_ACCUMULATE in the
 * plan, the frame's sums are added to vis; otherwise vis is overwritten.
 * The channel kernel (see xeng_plan_set_tuning) with S > 1 time slices keeps
 * the slices' partial outputs, S F N(N+1) int32, in plan-owned device memory
 * allocated on first use (grown, after the plan's last call, when S grows).
 * Errors: XENG_EINVAL (NULL plan or pointer, T < 1), XENG_EPLAN (N or F differ
 * from the plan, T > T_max), XENG_EOVERFLOW (T > XENG_T_EXACT_MAX),
 * XENG_ENOMEM (that memory cannot be allocated), XENG_EHIP.
 */
int xeng_correlate(xeng_plan_t p, const uint8_t *samples, int N, int F, int T,
                   int32_t *vis, void *stream);

/*
 * Tuning knobs of a plan (0 = choose automatically):
 *   split_t  number of time slices per tile (1 = one workgroup per tile; more
 *            slices fill the GPU when there are few tiles, at the price of
 *            exact integer atomic adds into vis, or, for the channel kernel,
 *            of partial outputs summed by a second kernel);
 *   kernel   tile shape: 1 = 128 x 128 baselines per workgroup (two
 *            workgroups per CU), 2 = 128 x 256 (one per CU; used only when
 *            N % 16 == 0 and the samples are 16-byte aligned, else 1),
 *            3 / 4 = 128 x 128 with the wave roles of diagonal tiles fixed:
 *            3 splits the sub-tile above the diagonal between two waves and
 *            skips the block below it, 4 keeps the off-diagonal roles (4
 *            applies to 16-byte-aligned frames without time shifting; others
 *            always split).  1 chooses the diagonal roles by N (split up to
 *            1024 inputs).  5 = the channel kernel: one workgroup of eight
 *            waves per (channel, time slice) covers the whole triangle of a
 *            channel of at most 256 inputs, each sample read once; several
 *            time slices store partial outputs that a second kernel sums
 *            into vis (int8 form only; the FP8 form, time shifting through
 *            the loads and N > 256 use 1).  Automatic: 5 for the int8 form at 128 < N <= 256 with
 *            N % 16 == 0 and 16-byte-aligned samples, else 1, the fastest on
 *            gfx950 at the measured sizes; the autotuner (tune.tune_plain)
 *            picks per shape.
 * Errors: XENG_EINVAL (NULL plan, negative split_t, kernel outside 0..5).
 */
int xeng_plan_set_tuning(xeng_plan_t p, int split_t, int kernel);

/*
 * Output gating (Sec. IV-C, "Output Gating"): the integration is partitioned
 * into G sub-buffers by the time of each sample, e.g. by the phase of a
 * pulsar's period or of an injected calibration signal, so that "on" and
 * "off" visibilities are formed within one integration.
 *
 * xeng_plan_gated: a plan as xeng_plan (same N, F, T_max, flags; it also
 * serves xeng_correlate) that can gate into up to G_max buffers.  It
 * allocates, once, pinned host staging and device tables for the runs of a
 * frame of T_max samples: about 8 (T_max + G_max) bytes of each.
 * Errors: as xeng_plan; XENG_EINVAL for G_max outside 1..XENG_G_MAX;
 * XENG_ENOMEM / XENG_EHIP when the tables cannot be allocated.
 *
 * xeng_correlate_gated: for every g in 0..G-1,
 *   vis[g][f][b(i,j)] = sum over t with gate[t] == g of x[t][f][i] conj(x[t][f][j])
 * (overwritten, or added with XENG_ACCUMULATE); samples whose gate is outside
 * 0..G-1 are dropped.
 *   gate   HOST array of T int32, read before the call returns.
 *   vis    device int32 [G][F][N(N+1)/2][2] (gate-major), caller-owned.
 * Asynchronous on `stream` like xeng_correlate.  The gate array becomes runs
 * of equal gate, uploaded from the plan's staging; a call first waits for the
 * previous call's upload to finish reading that staging.  Every (channel,
 * tile, gate) is one work item that integrates all runs of its gate: cost
 * grows with the number of runs only through their ragged edges (a run is
 * integrated in whole chunks of 64 samples, so runs shorter than 64 samples
 * are costly), and the output is written once.  A gate whose runs, rounded
 * up to whole chunks, hold more samples in one launch than one exact
 * integration may (XENG_F8_FLUSH_MAX in FP8, XENG_I8_SEG_MAX in int8) is
 * split into work items that add into its buffer with int32 atomics, so that
 * every sum stays exact however short the runs are.
 * Errors: XENG_EINVAL (NULL pointers, N, F, T or G < 1), XENG_EPLAN (not a
 * gated plan, G > G_max, N or F other than planned, T > T_max),
 * XENG_EOVERFLOW (T > XENG_T_EXACT_MAX), XENG_EHIP.
 */
int xeng_plan_gated(xeng_plan_t *out, int N, int F, int T_max, int G_max, unsigned flags);
int xeng_correlate_gated(xeng_plan_t p, const uint8_t *samples, int N, int F, int T,
                         const int32_t *gate, int G, int32_t *vis, void *stream);

/*
 * Time shifting (Sec. IV-C, "Time Shifting"): inputs from distant stations
 * decorrelate unless their samples are shifted in time.  After this call the
 * plan's correlations (xeng_correlate and xeng_correlate_gated) read input n
 * at time t - delays[n]:
 *   V_f[i][j] = sum_t x[t - d_i][f][i] conj(x[t - d_j][f][j]),
 * where rows t < 0 are the D_max rows of history the caller keeps in memory
 * directly before `samples` (e.g. the previous frame's tail in a ring of
 * frames); they must be readable, and they are read only for d > t.
 *   delays  HOST array of N ints in 0..D_max, one value per aligned group of
 *           16 inputs (the unit the kernels load); NULL turns shifting off.
 * Replacing delays first waits (on the host) for the plan's last call that
 * read them: an event recorded on that call's stream, not a device-wide sync.
 * Needs (D_max + 64) F N < 2^31.  The delays are copied (synchronously) to
 * plan-owned device memory.  The 128 x 256 tile kernel is not used while
 * shifting.  Delays equal within every aligned block of 128 inputs are
 * applied in the correlation's loads at almost no cost; delays that differ
 * inside a block make each call first copy the frame, shifted, into a
 * plan-owned buffer of T_max F N bytes (allocated here, once), which the
 * correlation then reads unshifted.
 * Errors: XENG_EINVAL (NULL plan, a delay outside 0..D_max, delays that differ
 * within a 16-input group, D_max too large), XENG_EPLAN (batch plan),
 * XENG_ENOMEM, XENG_EHIP.
 */
int xeng_plan_set_delays(xeng_plan_t p, const int32_t *delays, int D_max);

/*
 * Flagged data (Sec. IV-A, "Data Flow"): packets lost on the way from the
 * F-engine, and its flags for ADC saturation or channelizer overflow, mark
 * samples as invalid; the count of such data renormalises the integrated
 * matrices.  A flagged sample takes no part in the integration:
 *   vis[f][b(i,j)]    = sum over t with x[t][f][i] and x[t][f][j] both valid
 *                       of x_i conj(x_j),
 *   counts[f][b(i,j)] = the number of such t (int32 [F][N(N+1)/2]).
 *
 * xeng_plan_flagged: a plan as xeng_plan (it also serves xeng_correlate) that
 * owns the count workspace, allocated here: an event frame of T_max x F x N
 * bytes (as much as a frame), an int32 matrix of vis's size and about 12 F N
 * bytes of counters.
 * Errors: as xeng_plan; XENG_ENOMEM / XENG_EHIP when allocation fails.
 *
 * xeng_correlate_flagged:
 *   samples  device uint8 [T][F][N], MODIFIED: every flagged sample is set to
 *            0x88 (value 0) before the correlation reads the frame.
 *   flags    device uint32 [T][F][ceil(N / 32)]: bit (i % 32) of word i / 32
 *            set = sample (t, f, i) invalid; bits of inputs >= N are ignored.
 *   vis      as xeng_correlate; counts as above (both overwritten, or added to
 *            with XENG_ACCUMULATE).
 * Asynchronous on `stream`, with no host synchronisation.  Rows with one
 * invalid input are counted per input; rows with several become rows of an
 * event frame, which the int8 MFMA kernel correlates: identical rows within a
 * block of 64 (a saturated input, a lost packet) take one or two event rows,
 * distinct ones half a row each.  A frame whose rows all differ and all have
 * several invalid inputs costs about half a frame more.
 * Not available while time shifting is set (XENG_EPLAN).
 * Errors: XENG_EINVAL (NULL pointer, N, F or T < 1), XENG_EPLAN (not a flagged
 * plan, shifting set, N or F other than planned, T > T_max), XENG_EOVERFLOW,
 * XENG_EHIP.
 *
 * xeng_normalize: renormalised visibilities, float32 [F][N(N+1)/2][2],
 *   out = vis * scale / counts  (in float64, rounded once to float32),
 * and 0 where counts is 0.  scale = the number of samples integrated gives
 * the sums a loss-free integration would have had; scale = 1 the mean product
 * per valid sample.  N and F are the plan's; any single-instance plan serves.
 * Errors: XENG_EINVAL (NULL pointer, scale not finite and > 0), XENG_EPLAN
 * (batch plan), XENG_EHIP.
 */
int xeng_plan_flagged(xeng_plan_t *out, int N, int F, int T_max, unsigned flags);
int xeng_correlate_flagged(xeng_plan_t p, uint8_t *samples, const uint32_t *flags, int N, int F,
                           int T, int32_t *vis, int32_t *counts, void *stream);
int xeng_normalize(xeng_plan_t p, const int32_t *vis, const int32_t *counts, double scale,
                   float *out, void *stream);

/*
 * Discrete beamforming (Sec. IV-C, "Discrete Beamforming"): the data of all
 * inputs are phase-shifted and summed so that a signal from one direction adds
 * in phase, and the sum is written out at the sample cadence:
 *   beams[t][f][b] = sum over n of w[f][b][n] * x[t][f][n]
 * (complex; the weights are applied as given, without a conjugate: to point
 * at a direction, pass w = A e^{-i phi_n} rounded, with phi_n the phase of
 * that direction's signal at input n and A <= 127).  Exact in int32.
 *
 * xeng_plan_beams: a plan for B beams (1..XENG_BEAMS_MAX) over frames of N
 * inputs, F channels and T <= T_max samples; flags must be 0.  Needs
 * 515 F N + 256 < 2^31 (longer frames run as several launches).  Allocates the weight operands on the device:
 * 8 F ceil(N / 128) ceil(2B / 32) KiB.
 * Errors: XENG_EINVAL (out NULL, sizes out of range, flags), XENG_EOVERFLOW,
 * XENG_ENOMEM, XENG_EHIP.
 *
 * xeng_beam_set_weights: weights, HOST int8 [F][B][N][2] (re, im), each in
 * -127..127.  They are laid out for the matrix cores on the host and copied
 * (synchronously, after the plan's last xeng_beamform has finished reading the
 * previous weights) to plan-owned device memory; call again to re-point.
 * Errors: XENG_EINVAL (NULL, a weight of -128), XENG_EPLAN (not a beam
 * plan), XENG_EHIP.
 *
 * xeng_beamform: beams, device int32 [T][F][B][2] (re, im), from samples
 * [T][F][N] (device, layout above).  Asynchronous on `stream`.  Every sample
 * byte is read once per 64 beams (one launch covers up to 64 beams).
 * Errors: XENG_EINVAL (NULL pointer, sizes < 1), XENG_EPLAN (not a beam plan,
 * no weights set, N or F other than planned, T > T_max), XENG_EHIP.
 */
int xeng_plan_beams(xeng_plan_t *out, int N, int F, int T_max, int B, unsigned flags);
int xeng_beam_set_weights(xeng_plan_t p, const int8_t *weights);
int xeng_beamform(xeng_plan_t p, const uint8_t *samples, int N, int F, int T, int32_t *beams,
                  void *stream);

/* Free a plan (NULL is accepted).  Waits for nothing: the caller must not
 * destroy a plan with work still in flight on its stream. */
int xeng_destroy(xeng_plan_t p);

/* Text of the last XENG_EHIP error seen by this plan ("" if none). */
const char *xeng_plan_error(xeng_plan_t p);

/* ------------------------------------------------------------------------
 * Batched form: many independent correlation instances in one launch.
 * Each instance has its own N, F and T, its own samples and its own vis, laid
 * out as above.  Channels of different instances never mix: this is the same
 * definition applied instance by instance.
 */
typedef struct xeng_instance {
    int N;       /* inputs */
    int F;       /* channels */
    int T;       /* samples integrated per call */
    int split_t; /* time slices per tile; 0 = automatic: one count for all such instances,
                    chosen from the whole batch's tiles (autotuner output goes here) */
} xeng_instance;

/*
 * Plan a batch of `count` instances (copied; descs may be freed after the
 * call).  Each instance is the correlation of xeng_correlate (Sec. IV-C,
 * "Full Correlation"; Eq. (1)) on its own frame.  flags as for xeng_plan (the form applies to every instance), plus
 * XENG_SHARED_VIS, which needs XENG_ACCUMULATE.  The plan owns a device table
 * of work items, built on first use.
 * Errors: XENG_EINVAL (out or descs NULL, count < 1, any N, F or T < 1,
 * any N > XENG_N_MAX, negative split_t, unknown flags, XENG_SHARED_VIS without
 * XENG_ACCUMULATE), XENG_EOVERFLOW (any T > XENG_T_EXACT_MAX), XENG_ENOMEM.
 */
int xeng_plan_batch(xeng_plan_t *out, const xeng_instance *descs, int count, unsigned flags);

/*
 * Correlate every instance of a batch plan (the definition of
 * xeng_correlate, Sec. IV-C "Full Correlation", per instance): samples[k] and
 * vis[k] are the device buffers of instance k (host arrays of count device pointers).  One
 * persistent kernel launch covers all instances.  An instance whose samples[k]
 * is NULL is skipped by this call (its vis[k] is ignored and untouched), so a
 * plan over a pool of slots serves any subset of them.  Pointers are copied to
 * the device through plan-owned pinned staging on the given stream (a ring
 * of four copies); the call waits on the host only when the pointers changed
 * and the staging copy it reuses still holds an upload four calls old that
 * has not run yet.
 * Errors: XENG_EINVAL (NULL plan or arrays, NULL vis[k] of an active
 * instance), XENG_EPLAN (not a batch plan), XENG_EHIP, XENG_ENOMEM.
 */
int xeng_correlate_batch(xeng_plan_t p, const uint8_t *const *samples, int32_t *const *vis,
                         void *stream);

/*
 * As xeng_correlate_batch, replaying a HIP graph captured on the first call
 * for this exact array of pointers (re-captured when any pointer changes).
 * For fixed slot buffers, a call is one hipGraphLaunch.
 */
int xeng_correlate_batch_graph(xeng_plan_t p, const uint8_t *const *samples,
                               int32_t *const *vis, void *stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the batched form without a
 * plan.  The result is that of xeng_plan_batch(descs, count, flags) followed
 * by xeng_correlate_batch(samples, vis) on `stream`; instances with
 * samples[k] == NULL are skipped.  The call only launches kernels: no
 * allocation, no copy, no host synchronisation.  The instance table, the work
 * list and the work counter live in the library's fixed device workspace, a
 * file-scope array of about 2 MiB that each GPU the library runs on holds
 * until the process ends; the call's first use on a device looks up its
 * address there.  Every call on a GPU shares that GPU's workspace: calls that
 * overlap on one GPU (on several streams, or from several threads) race, and
 * the caller must order them (one stream, or events).
 * Limits: at most XENG_NOALLOC_INST_MAX active instances and at most
 * XENG_NOALLOC_ITEMS_MAX work items, the sum over active instances of
 * F x nt (nt + 1) / 2 x (time slices), nt = ceil(N / 128).
 * Errors: XENG_EINVAL (NULL arrays, count < 1, any N, F or T < 1, any
 * N > XENG_N_MAX, negative split_t, unknown flags, XENG_SHARED_VIS without
 * XENG_ACCUMULATE, NULL vis[k] of an active instance), XENG_EOVERFLOW (any
 * T > XENG_T_EXACT_MAX), XENG_ELIMIT (a limit above is exceeded; nothing is
 * queued), XENG_EHIP (a HIP runtime or launch error; with no plan, its text
 * is not kept).
 */
int xeng_correlate_batch_noalloc(const xeng_instance *descs, int count, unsigned flags,
                                 const uint8_t *const *samples, int32_t *const *vis,
                                 void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XENG_H */
