// The channel kernel: one workgroup of eight waves correlates every baseline
// of a channel of at most 256 inputs over one time slice (Sec. IV-C, "Full
// Correlation"; the N(N+1)/2 baselines of Eq. (1), e.g. the 32,896 of the
// 256-input Pathfinder of Sec. II), reading each sample of the slice once.
//
// Work split.  The 256 inputs form eight 32-input fragments (one MFMA block
// edge) and four 64-input quarters q = 0..3; quarter q lies in block q / 2 of
// the stage at column 64 (q % 2).  The triangle holds 28 blocks off the
// diagonal and 8 on it.  An off-diagonal block takes two accumulators (Re and
// Im, as in the tile kernels); a diagonal block takes one (see DiagRole), so
// the channel is 28 x 2 + 8 = 64 accumulators of 16 registers, eight per
// wave, and every wave issues the same number of MFMAs:
//
//   waves 0..5  the six off-diagonal 64 x 64 quarter pairs (QA, QB), QA < QB,
//               2 x 2 blocks each (OffRole);
//   waves 6, 7  quarters 0, 1 and 2, 3: per quarter, its block between its
//               two fragments (Re, Im) and its two diagonal blocks (DiagRole).
//
// Each wave also keeps the code sums of one fragment (the offset corrections;
// see TileSums), so that the eight waves cover the 256 inputs once.
//
// Staging.  Every fragment is read by four waves, so its nibbles are split
// once, by the thread that stages them: a stage holds, per 128-input block,
// a plane of real codes and a plane of imaginary codes (rows = times, as
// loaded, one code a byte; PROW-byte rows as in xcorr_tile.hpp).  A fragment
// read is then two transpose reads, which deliver the operand [m(8), r(8)]
// with no arithmetic.
//
// The workgroup (512 threads, up to 256 registers a thread, 86 KiB of LDS)
// fills a CU; a launch is one workgroup per (channel, time slice).  With
// several slices, each stores its own partial triangles and
// chan_reduce_kernel sums them into vis.
#include "xcorr_device.hpp"
#include "xeng_chan.hpp"

namespace xeng {

namespace {

constexpr int CH_THREADS = 512;
constexpr int CH_IN = 2 * BT;  // inputs a workgroup covers
// a stage: the real and imaginary code planes of blocks 0 and 1 (block b,
// part p at (2 b + p) PLANE)
constexpr int CH_STAGE = 4 * PLANE;
// epilogue LDS beyond the two stages: per-lane partial sums part[half][plane][256]
// and the per-input code sums S[256] (int2: real, imaginary)
constexpr int CH_PART = 2 * CH_STAGE;
constexpr int CH_SUMS = CH_PART + 2 * 2 * CH_IN * 4;
constexpr int CH_LDS = CH_SUMS + CH_IN * 8;
// a diagonal block as a 32 x 33 int matrix (one pad column), for its transpose
constexpr int CH_DIAG = 32 * 33 * 4;
static_assert(2 * 4 * CH_DIAG <= 2 * CH_STAGE, "the diagonal blocks of two waves fit the stages");
static_assert(256 * PROW <= CH_STAGE, "the sums slots lie in the first stage");

// first byte of quarter q's real codes within a stage (its imaginary codes
// follow PLANE bytes later)
constexpr int qoff(int q) { return (q >> 1) * 2 * PLANE + 64 * (q & 1); }

// Staging role: every thread loads and stores two 16-byte row pieces of a
// chunk, sixteen inputs 16 seg.. of plane 0 and of plane 1 at one time `row`.
// Rows follow q = tid / 8 as 0, 4, 1, 5, 2, 6, 3, 7, 8, 12, ..., so that eight
// lanes read one 128-byte row and sixteen lanes write two plane rows 4 apart
// (all 64 LDS banks once).
struct ChanStage {
  int row, seg;
  __device__ __forceinline__ explicit ChanStage(int tid) : seg(tid & 7) {
    const int q = tid >> 3;
    row = 4 * (q & 1) + ((q >> 1) & 3) + 8 * (q >> 3);
  }
};

// Fast loads: both pieces inside the frame (N % 16 == 0, rows 16-byte
// aligned, F N <= 2^25 so that the offsets of 64 rows fit 31 bits).  `rows`
// is the chunk's first row of the channel (uniform).  Inputs at or past N
// read input 0 instead: their plane columns only reach baselines past N,
// which are never written.
__device__ __forceinline__ void chan_load_fast(v4i (&raw)[2], const uint8_t* rows, uint32_t off0,
                                               uint32_t off1) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)rows, (short)0, 0x7fffffff, 0x00020000);
  raw[0] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off0, 0, 0));
  raw[1] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off1, 0, 0));
}

// General loads (frame edges, ragged tails, unaligned frames): absent samples
// and inputs read as the code of 0 + 0i.
__device__ __forceinline__ void chan_load_edge(v4i (&raw)[2], const uint8_t* samples,
                                               long long row_stride, int f, int N,
                                               const ChanStage& st, int t_chunk, int t_end) {
  raw[0] = load_piece_edge(samples, row_stride, f, N, 16 * st.seg, t_chunk + st.row, t_end);
  raw[1] = load_piece_edge(samples, row_stride, f, N, BT + 16 * st.seg, t_chunk + st.row, t_end);
}

// Piece k (block k) of a thread: its real (high nibble) and imaginary (low
// nibble) codes into the block's two planes.
__device__ __forceinline__ void chan_stage_piece(const v4i& raw, int k, uint8_t* stage,
                                                 const ChanStage& st) {
  const uint32_t c = 0x0F0F0F0Fu;
  const v4i r = v4i{(int)(((uint32_t)raw.x >> 4) & c), (int)(((uint32_t)raw.y >> 4) & c),
                    (int)(((uint32_t)raw.z >> 4) & c), (int)(((uint32_t)raw.w >> 4) & c)};
  const v4i m = v4i{(int)((uint32_t)raw.x & c), (int)((uint32_t)raw.y & c),
                    (int)((uint32_t)raw.z & c), (int)((uint32_t)raw.w & c)};
  uint8_t* d = stage + 2 * k * PLANE + st.row * PROW + 16 * st.seg;
  *reinterpret_cast<v4i*>(d) = r;
  *reinterpret_cast<v4i*>(d + PLANE) = m;
}

// The codes of one fragment read: lane l holds input l % 32 of the fragment
// at eight times (the half l / 32 of the k-step's sixteen).  p: the
// fragment's real codes at the k-step.
struct Frag {
  v2i r, m;
};

__device__ __forceinline__ Frag frag_read(const uint8_t* p) {
  return Frag{lds_tr8(p), lds_tr8(p + PLANE)};
}

// Operand [m(8), r(8)]: Re = A_i . A_j (see compute_chunk).
__device__ __forceinline__ v4i op_a(const Frag& x) { return v4i{x.m.x, x.m.y, x.r.x, x.r.y}; }

// Bytewise code sums of one fragment (at most 16 codes a byte between
// flushes), folded into the thread's LDS slot (see sum_slot) by chan_flush.
struct ChanSums {
  uint32_t r, m;
};

__device__ __forceinline__ void chan_add(ChanSums& sm, const Frag& x) {
  sm.r = badd(x.r.x, x.r.y, sm.r);
  sm.m = badd(x.m.x, x.m.y, sm.m);
}

__device__ __forceinline__ void chan_flush(ChanSums& sm, uint8_t* lds) {
  uint32_t* p = sum_slot(lds);
  atomicAdd(p + 0, __builtin_amdgcn_udot4(sm.r, 0x01010101u, 0u, false));
  atomicAdd(p + 1, __builtin_amdgcn_udot4(sm.m, 0x01010101u, 0u, false));
  sm.r = sm.m = 0u;
}

// Everything the epilogue needs to turn sums of codes into visibilities.
struct ChanOut {
  int32_t* base;  // the channel's packed triangle
  int N, teff;
  const int2* S;  // per-input code sums (LDS)
};

// Row of register v in a lane's share of a 32 x 32 MFMA block (its column is
// lane % 32).
__device__ __forceinline__ int blk_row(int v, int lane) {
  return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
}

// A lane's share of a block, (vr, vi) of baselines (i0 + blk_row(v), j) for
// the v set in `ok`, into vis in write mode MODE (see put_pairs).
template <int MODE>
__device__ __forceinline__ void store16(const ChanOut& o, int i0, int j, int lane,
                                        const int (&vr)[16], const int (&vi)[16], uint32_t ok) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int b[8], r[8], m[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      b[u] = pair_index(i0 + blk_row(8 * h + u, lane), j, o.N);
      r[u] = vr[8 * h + u];
      m[u] = vi[8 * h + u];
    }
    put_pairs<MODE>(o.base, b, r, m, (ok >> (8 * h)) & 0xFFu);
  }
}

// Write an off-diagonal block (rows i0.., columns j0.., j > i throughout):
// re = sum A_i A_j and im = sum A_i Y_j of codes, with Y = [r, 15 - m], so
//   Re V = re - 8 (Sr_i + Sm_i + Sr_j + Sm_j) + 128 T,
//   Im V = im - 15 Sr_i - 8 (Sm_i - Sr_i) + 8 (Sm_j - Sr_j)
// (the code offsets of 8, see stage_piece and row_corr / col_corr).
template <int MODE>
__device__ __forceinline__ void write_off(const ChanOut& o, int i0, int j0, const v16i& re,
                                          const v16i& im, int lane) {
  const int j = j0 + (lane & 31);
  if (j >= o.N) return;
  const int2 sj = o.S[j];
  int vr[16], vi[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int2 si = o.S[i0 + blk_row(v, lane)];
    vr[v] = re[v] + 128 * o.teff - 8 * (si.x + si.y + sj.x + sj.y);
    vi[v] = im[v] - 15 * si.x - 8 * (si.y - si.x) + 8 * (sj.y - sj.x);
  }
  store16<MODE>(o, i0, j, lane, vr, vi, 0xFFFFu);
}

// Write a diagonal block (inputs n0..n0+31) from its one accumulator
//   D_ij = sum_t A_i . Z_j,  Z = [m + r, r + 15 - m]
//        = Re_ij + Im_ij + 15 Sr_i            (sums of codes)
// and its transpose D_ji = Re_ij - Im_ij + 15 Sr_j (Re is symmetric, Im
// antisymmetric): Re_ij = (D_ij + D_ji - 15 (Sr_i + Sr_j)) / 2 and
// Im_ij = (D_ij - D_ji - 15 (Sr_i - Sr_j)) / 2, both exact (even numerators).
// The transpose comes through the LDS matrix `m` (32 x 33 ints, this wave's).
template <int MODE>
__device__ __forceinline__ void write_diag(const ChanOut& o, int n0, const v16i& d, int* m,
                                           int lane) {
  const int lj = lane & 31;
#pragma unroll
  for (int v = 0; v < 16; ++v) m[blk_row(v, lane) * 33 + lj] = d[v];
  // a wave's LDS operations complete in order: its writes land before its reads
  const int j = n0 + lj;
  if (j >= o.N) return;
  const int2 sj = o.S[j];
  int vr[16], vi[16];
  uint32_t ok = 0u;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int di = blk_row(v, lane), i = n0 + di;
    const int dt = m[lj * 33 + di];
    const int2 si = o.S[i];
    const int re = (d[v] + dt - 15 * (si.x + sj.x)) >> 1;
    const int im = (d[v] - dt - 15 * (si.x - sj.x)) >> 1;
    vr[v] = re + 128 * o.teff - 8 * (si.x + si.y + sj.x + sj.y);
    vi[v] = i == j ? 0 : im - 8 * (si.y - si.x) + 8 * (sj.y - sj.x);
    ok |= (uint32_t)(i <= j) << v;
  }
  store16<MODE>(o, n0, j, lane, vr, vi, ok);
}

// Off-diagonal quarter pair (QA, QB): blocks (a, b) between fragment a of QA
// and fragment b of QB.  SUM: the fragment whose codes it sums, 0 / 1 = A
// fragment a, 2 / 3 = B fragment b - 2.
template <int QA, int QB, int SUM>
struct OffRole {
  static constexpr int kSumFrag = SUM < 2 ? 2 * QA + SUM : 2 * QB + SUM - 2;
  v16i re[2][2], im[2][2];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) re[a][b] = im[a][b] = v16i{};
  }

  // One chunk from the stage at `cur`; with `stg`, the next chunk's two
  // pieces are stored into the stage at `nxt` between the k-steps.  The
  // fragments of k-step s + 1 are read before the MFMAs of k-step s, so that
  // the transpose reads run under the matrix work (both waves of a SIMD
  // belong to this workgroup and reach each barrier together: neither hides
  // the other's LDS latency).
  __device__ __forceinline__ void chunk(const uint8_t* cur, int lane_rd, ChanSums& sm,
                                        const v4i* stg, uint8_t* nxt, const ChanStage& st) {
    const uint8_t* pa = cur + qoff(QA) + lane_rd;
    const uint8_t* pb = cur + qoff(QB) + lane_rd;
    Frag fa[2][2], fb[2][2];  // [k-step parity][fragment]
    auto read = [&](int s, Frag (&ga)[2], Frag (&gb)[2]) {
#pragma unroll
      for (int a = 0; a < 2; ++a) ga[a] = frag_read(pa + 16 * s * PROW + 32 * a);
#pragma unroll
      for (int b = 0; b < 2; ++b) gb[b] = frag_read(pb + 16 * s * PROW + 32 * b);
    };
    read(0, fa[0], fb[0]);
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      const int q = s & 1;
      if (s + 1 < KC / 16) read(s + 1, fa[q ^ 1], fb[q ^ 1]);
      // keep the reads ahead of this k-step's MFMAs (the scheduler would sink
      // them to their use to save registers)
      __builtin_amdgcn_sched_barrier(0);
      v4i A[2], B[2], Y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        A[a] = op_a(fa[q][a]);
        if (SUM == a) chan_add(sm, fa[q][a]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Frag& x = fb[q][b];
        const int c15 = 0x0F0F0F0F;
        // B = [m, r] and Y = [r, 15 - m] share registers
        const v8i w = v8i{x.m.x, x.m.y, x.r.x, x.r.y, x.m.x ^ c15, x.m.y ^ c15, 0, 0};
        B[b] = __builtin_shufflevector(w, w, 0, 1, 2, 3);
        Y[b] = __builtin_shufflevector(w, w, 2, 3, 4, 5);
        if (SUM == 2 + b) chan_add(sm, x);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          re[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], B[b], re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], Y[b], im[a][b], 0, 0, 0);
        }
      if (stg && (s & 1) == 0) chan_stage_piece(stg[s >> 1], s >> 1, nxt, st);
    }
  }

  template <int MODE>
  __device__ __forceinline__ void write(const ChanOut& o, int*, int lane) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i0 = 64 * QA + 32 * a, j0 = 64 * QB + 32 * b;
        if (i0 < o.N && j0 < o.N) write_off<MODE>(o, i0, j0, re[a][b], im[a][b], lane);
      }
  }
};

// Quarters D0 and D0 + 1 with their diagonal blocks.  Per quarter e, with
// fragments P (its first 32 inputs) and Q: acc[e][0] = D of block (P, P),
// acc[e][1] = D of (Q, Q), acc[e][2] / [3] = Re / Im of block (P, Q).  SUM:
// the fragment (0..3 = P0, Q0, P1, Q1) whose codes it sums.
template <int D0, int SUM>
struct DiagRole {
  static constexpr int kSumFrag = 2 * D0 + SUM;
  v16i acc[2][4];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[e][k] = v16i{};
  }

  // One chunk (see OffRole::chunk; the fragments of k-step s + 1 are read
  // before the MFMAs of k-step s).
  __device__ __forceinline__ void chunk(const uint8_t* cur, int lane_rd, ChanSums& sm,
                                        const v4i* stg, uint8_t* nxt, const ChanStage& st) {
    Frag fr[2][2][2];  // [k-step parity][quarter e][P, Q]
    auto read = [&](int s, Frag (&g)[2][2]) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint8_t* p = cur + qoff(D0 + e) + lane_rd + 16 * s * PROW;
        g[e][0] = frag_read(p);
        g[e][1] = frag_read(p + 32);
      }
    };
    read(0, fr[0]);
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      const int q = s & 1;
      if (s + 1 < KC / 16) read(s + 1, fr[q ^ 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const Frag& P = fr[q][e][0];
        const Frag& Q = fr[q][e][1];
        if (SUM == 2 * e) chan_add(sm, P);
        if (SUM == 2 * e + 1) chan_add(sm, Q);
        const int c15 = 0x0F0F0F0F;
        const v4i AP = op_a(P), AQ = op_a(Q);
        // Z = [m + r, r + 15 - m]: bytes stay in 0..30, no carry between them
        const v4i ZP = v4i{P.m.x + P.r.x, P.m.y + P.r.y, P.r.x + (P.m.x ^ c15),
                           P.r.y + (P.m.y ^ c15)};
        const v4i ZQ = v4i{Q.m.x + Q.r.x, Q.m.y + Q.r.y, Q.r.x + (Q.m.x ^ c15),
                           Q.r.y + (Q.m.y ^ c15)};
        const v4i YQ = v4i{Q.r.x, Q.r.y, Q.m.x ^ c15, Q.m.y ^ c15};
        acc[e][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(AP, ZP, acc[e][0], 0, 0, 0);
        acc[e][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(AQ, ZQ, acc[e][1], 0, 0, 0);
        acc[e][2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(AP, AQ, acc[e][2], 0, 0, 0);
        acc[e][3] = __builtin_amdgcn_mfma_i32_32x32x32_i8(AP, YQ, acc[e][3], 0, 0, 0);
      }
      if (stg && (s & 1) == 0) chan_stage_piece(stg[s >> 1], s >> 1, nxt, st);
    }
  }

  // m: this wave's four transpose matrices (CH_DIAG bytes each)
  template <int MODE>
  __device__ __forceinline__ void write(const ChanOut& o, int* m, int lane) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int n0 = 64 * (D0 + e);
      if (n0 >= o.N) continue;
      write_diag<MODE>(o, n0, acc[e][0], m + (2 * e) * (CH_DIAG / 4), lane);
      if (n0 + 32 < o.N) {
        write_diag<MODE>(o, n0 + 32, acc[e][1], m + (2 * e + 1) * (CH_DIAG / 4), lane);
        write_off<MODE>(o, n0, n0 + 32, acc[e][2], acc[e][3], lane);
      }
    }
  }
};

// Per-thread loop state.
struct ChanCtx {
  ChanStage st;
  uint32_t off0, off1;  // fast-load offsets of the two pieces (row and inputs)
  int lane_rd;
  ChanSums sm;
  __device__ __forceinline__ explicit ChanCtx(int tid) : st(tid) {}
};

// One steady step: load chunk `ld_chunk` into `ld`, compute the chunk at
// `cur` while storing `stg` (the next chunk) into `nxt`, then synchronise.
template <class R>
__device__ __forceinline__ void chan_step(R& role, ChanCtx& x, const uint8_t* rows,
                                          long long row_stride, uint8_t* lds, int cur, int nxt,
                                          const v4i (&stg)[2], v4i (&ld)[2], int ld_chunk) {
  chan_load_fast(ld, rows + (long long)ld_chunk * KC * row_stride, x.off0, x.off1);
  __builtin_amdgcn_sched_barrier(0);
  role.chunk(lds + cur, x.lane_rd, x.sm, stg, lds + nxt, x.st);
  __syncthreads();
}

// The chunks of [t_begin, t_end): a steady state over whole chunks inside the
// frame, in groups of four, with loads three chunks ahead (four register
// sets of two pieces: the set of chunk c + 3 loads while chunk c computes and
// chunk c + 1 is stored), then a general loop for the rest.  Loads past the
// last fast chunk reload it; what they stage is never computed.  Returns the
// samples integrated, padding of a ragged last chunk included.
template <bool ALIGNED, class R>
__device__ __forceinline__ int chan_range(R& role, ChanCtx& x, const uint8_t* samples,
                                          long long row_stride, int N, int f, int t_begin,
                                          int t_end, uint8_t* lds) {
  const int len = t_end > t_begin ? t_end - t_begin : 0;
  const int nchunks = (len + KC - 1) / KC;
  const uint8_t* rows = samples + (long long)t_begin * row_stride + (long long)f * N;
  constexpr int B0 = 0, B1 = CH_STAGE;
  const int nfast = ALIGNED ? len / KC : 0;
  const int nsteady = nfast & ~3;
  int c = 0;
  if (nsteady >= 4) {
    v4i r0[2], r1[2], r2[2], r3[2];
    chan_load_fast(r0, rows, x.off0, x.off1);
    chan_load_fast(r1, rows + (long long)KC * row_stride, x.off0, x.off1);
    chan_load_fast(r2, rows + (long long)2 * KC * row_stride, x.off0, x.off1);
    chan_stage_piece(r0[0], 0, lds + B0, x.st);
    chan_stage_piece(r0[1], 1, lds + B0, x.st);
    __syncthreads();
    const int last = nfast - 1;
    for (; c < nsteady; c += 4) {
      chan_step(role, x, rows, row_stride, lds, B0, B1, r1, r3, min(c + 3, last));
      chan_step(role, x, rows, row_stride, lds, B1, B0, r2, r0, min(c + 4, last));
      chan_flush(x.sm, lds);
      chan_step(role, x, rows, row_stride, lds, B0, B1, r3, r1, min(c + 5, last));
      chan_step(role, x, rows, row_stride, lds, B1, B0, r0, r2, min(c + 6, last));
      chan_flush(x.sm, lds);
    }
  }
  v4i raw[2];
  auto load = [&](int cc) {
    if (ALIGNED && (cc + 1) * KC <= len)
      chan_load_fast(raw, rows + (long long)cc * KC * row_stride, x.off0, x.off1);
    else
      chan_load_edge(raw, samples, row_stride, f, N, x.st, t_begin + cc * KC, t_end);
  };
  if (c < nchunks) {
    load(c);
    chan_stage_piece(raw[0], 0, lds + (c & 1) * CH_STAGE, x.st);
    chan_stage_piece(raw[1], 1, lds + (c & 1) * CH_STAGE, x.st);
    __syncthreads();
  }
  for (; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    role.chunk(lds + (c & 1) * CH_STAGE, x.lane_rd, x.sm, nullptr, nullptr, x.st);
    chan_flush(x.sm, lds);
    if (more) {
      chan_stage_piece(raw[0], 0, lds + ((c + 1) & 1) * CH_STAGE, x.st);
      chan_stage_piece(raw[1], 1, lds + ((c + 1) & 1) * CH_STAGE, x.st);
    }
    __syncthreads();
  }
  return nchunks * KC;
}

// The whole work of one wave role: chunks, sums, epilogue.
template <bool ALIGNED, class R>
__device__ __forceinline__ void chan_wave(const ChanArgs& a, int f, int slice, int t_begin,
                                          int t_end, int wave, uint8_t* lds) {
  const int tid = threadIdx.x, lane = tid & 63;
  R role;
  role.clear();
  ChanCtx x(tid);
  const int n0 = 16 * x.st.seg, n1 = BT + 16 * x.st.seg;
  x.off0 = (uint32_t)x.st.row * (uint32_t)a.row_stride + (uint32_t)(n0 < a.N ? n0 : 0);
  x.off1 = (uint32_t)x.st.row * (uint32_t)a.row_stride + (uint32_t)(n1 < a.N ? n1 : 0);
  x.lane_rd = lane_read_offset<FORM_I8>(lane);
  x.sm = ChanSums{0u, 0u};
  // this thread's sums slot (it alone adds to it; the slot rows' bytes
  // 128..159 are never staged into)
  *reinterpret_cast<v4i*>(sum_slot(lds)) = v4i{0, 0, 0, 0};

  const int teff =
      chan_range<ALIGNED>(role, x, a.samples, a.row_stride, a.N, f, t_begin, t_end, lds);
  if (t_end <= t_begin) __syncthreads();  // every slot is cleared before it is read

  // per-input sums: lane l of the wave holds input 32 kSumFrag + l % 32 over
  // the half l / 32 of every k-step's samples
  int* part = reinterpret_cast<int*>(lds + CH_PART);
  int2* S = reinterpret_cast<int2*>(lds + CH_SUMS);
  {
    const v4i s = *reinterpret_cast<const v4i*>(sum_slot(lds));
    const int n = 32 * R::kSumFrag + (lane & 31), h = lane >> 5;
    part[(h * 2 + 0) * CH_IN + n] = s.x;
    part[(h * 2 + 1) * CH_IN + n] = s.y;
  }
  __syncthreads();  // partial sums complete, every slot read
  if (tid < CH_IN)
    S[tid] = make_int2(part[0 * CH_IN + tid] + part[2 * CH_IN + tid],
                       part[1 * CH_IN + tid] + part[3 * CH_IN + tid]);
  __syncthreads();
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  int32_t* out = a.partial ? a.partial + 2 * NB * ((long long)slice * a.F) : a.vis;
  ChanOut o{out + 2 * (long long)f * NB, a.N, teff, S};
  // waves 6 and 7 transpose their diagonal blocks through the (free) stages
  int* m = reinterpret_cast<int*>(lds) + (wave & 1) * 4 * (CH_DIAG / 4);
  // one dispatch on the (uniform) write mode: a lone slice stores or adds into
  // vis, several slices store into their own partial triangles
  if (a.write_mode == WM_ADD)
    role.template write<WM_ADD>(o, m, lane);
  else
    role.template write<WM_STORE>(o, m, lane);
}

}  // namespace

template <bool ALIGNED>
__global__ void __launch_bounds__(CH_THREADS, 1) xcorr_chan_kernel(ChanArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[CH_LDS];
  const int b = blockIdx.x;
  const int s = b % a.nslices, f = b / a.nslices;
  const int t_begin = a.t0 + s * a.slice_len;
  const int t_end = min(a.t1, t_begin + a.slice_len);
  // uniform per wave: the role dispatch is a scalar branch
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  switch (wave) {
    case 0: chan_wave<ALIGNED, OffRole<0, 1, 0>>(a, f, s, t_begin, t_end, wave, lds); break;
    case 1: chan_wave<ALIGNED, OffRole<0, 2, 1>>(a, f, s, t_begin, t_end, wave, lds); break;
    case 2: chan_wave<ALIGNED, OffRole<0, 3, 2>>(a, f, s, t_begin, t_end, wave, lds); break;
    case 3: chan_wave<ALIGNED, OffRole<1, 2, 0>>(a, f, s, t_begin, t_end, wave, lds); break;
    case 4: chan_wave<ALIGNED, OffRole<1, 3, 3>>(a, f, s, t_begin, t_end, wave, lds); break;
    case 5: chan_wave<ALIGNED, OffRole<2, 3, 0>>(a, f, s, t_begin, t_end, wave, lds); break;
    case 6: chan_wave<ALIGNED, DiagRole<0, 3>>(a, f, s, t_begin, t_end, wave, lds); break;
    default: chan_wave<ALIGNED, DiagRole<2, 1>>(a, f, s, t_begin, t_end, wave, lds); break;
  }
}

// The slices' partial triangles summed into vis: one pass over HBM, which
// costs less than the slices adding into vis with atomics after a fill (every
// workgroup of the channel kernel finishes at once, so nothing would hide the
// atomics).
__global__ void chan_reduce_kernel(const int32_t* __restrict__ part, int32_t* __restrict__ vis,
                                   long long n, int ns, int add) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if ((n & 3) == 0 && !(reinterpret_cast<uintptr_t>(vis) & 15)) {
    const long long n4 = n >> 2;
    const v4i* p4 = reinterpret_cast<const v4i*>(part);
    v4i* v4 = reinterpret_cast<v4i*>(vis);
    for (; i < n4; i += stride) {
      v4i acc = p4[i];
      for (int s = 1; s < ns; ++s) acc += p4[s * n4 + i];
      if (add) acc += v4[i];
      v4[i] = acc;
    }
  } else {
    for (; i < n; i += stride) {
      int acc = part[i];
      for (int s = 1; s < ns; ++s) acc += part[s * n + i];
      vis[i] = add ? vis[i] + acc : acc;
    }
  }
}

hipError_t launch_chan_reduce(const int32_t* partial, int32_t* vis, long long n, int ns, bool add,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (ns < 1) return hipErrorInvalidValue;
  long long blocks = ((n >> 2) + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  hipLaunchKernelGGL(chan_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, partial,
                     vis, n, ns, add ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_chan(const ChanArgs& a, bool aligned, hipStream_t stream) {
  if (a.N < 1 || a.N > CH_IN || a.nslices < 1 || a.slice_len < 1) return hipErrorInvalidValue;
  const long long grid = (long long)a.F * a.nslices;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid), blk(CH_THREADS);
  if (aligned)
    hipLaunchKernelGGL(xcorr_chan_kernel<true>, g, blk, 0, stream, a);
  else
    hipLaunchKernelGGL(xcorr_chan_kernel<false>, g, blk, 0, stream, a);
  return hipGetLastError();
}

}  // namespace xeng
