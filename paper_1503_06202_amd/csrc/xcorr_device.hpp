// Device code of the X-engine's 128 x 128 tile kernels for gfx950: staging,
// MFMA chunks, per-input sums and the tile body shared by the plain, gated and
// batched kernels (one workgroup per channel, tile of 128 x 128 baselines and
// time range; int8 or FP8 MFMA).
//
// What is computed: V_f[i][j] = sum_t x_i conj(x_j) over the upper triangle
// including the diagonal (Sec. I; Sec. IV-C, "Full Correlation"; the baseline
// count N(N+1)/2 of Eq. (1)), on 4+4-bit offset-binary samples (Sec. II-A,
// footnote).  The tile layout, the operand packing and the MFMA formulation are
// described in xcorr_tile.hpp.
#pragma once

#include <type_traits>

#include "xcorr_tile.hpp"
#include "xeng_internal.hpp"

namespace xeng {

// Staging role of a thread.  Every thread stages four 16-byte row pieces of a
// chunk (sixteen inputs at one time): pieces 0, 1 of the I block at times
// rI, rI + 16 and pieces 2, 3 of the J block at times rJ, rJ + 16, with
// rI = r0 + 32 h and rJ = r0 + 32 (1 - h) for the thread's half h of the
// workgroup, so that every thread does the same work.  The inputs are
// 16*seg.. of each block; r0 runs over 0..15 as q = (tid & 127) >> 3 does, in
// the order 0,4,1,5,2,6,3,7,8,12,9,13,10,14,11,15.  Eight consecutive lanes
// read one 128-byte row; sixteen consecutive lanes write two plane rows 4
// apart.
struct StageRole {
  int seg, rI, rJ;
  __device__ __forceinline__ explicit StageRole(int tid) : seg(tid & 7) {
    const int q = (tid & 127) >> 3, h = tid >> 7;
    const int r0 = 4 * (q & 1) + ((q >> 1) & 3) + 8 * (q >> 3);
    rI = r0 + 32 * h;
    rJ = r0 + 32 * (1 - h);
  }
};

// Fast path: the four pieces lie inside the frame.  `rows` points at the
// chunk's first row of this channel (uniform across the workgroup); offI /
// offJ add the thread's first I / J row and its inputs.  Buffer loads: the
// chunk's base goes into a scalar resource and the row offset of the second
// piece into the scalar offset, so that a thread keeps two 32-bit offsets
// instead of 64-bit addresses.  The host keeps F N <= 2^25 on this path, so
// every offset (at most 64 rows of F N bytes) stays below 2^31.
//
// Time shifting: the I and J pieces are read `shiftI` / `shiftJ` bytes (the
// largest delay of the block, in rows) before `rows`, and a lane's offset
// adds back its own segment's rows (see tile_body).
//
// NP: pieces per thread, 4 (I and J blocks) or 2 (the I block alone, for a
// diagonal tile, whose J block is the same rows).
template <int NP>
__device__ __forceinline__ void load_pieces_fast(v4i (&raw)[4], const uint8_t* __restrict__ rows,
                                                 long long row_stride, uint32_t offI,
                                                 uint32_t offJ, long long shiftI = 0,
                                                 long long shiftJ = 0) {
  const __amdgpu_buffer_rsrc_t rI =
      __builtin_amdgcn_make_buffer_rsrc((void*)(rows - shiftI), (short)0, 0x7fffffff, 0x00020000);
  const int s16 = (int)(16 * row_stride);
  raw[0] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rI, (int)offI, 0, 0));
  raw[1] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rI, (int)offI, s16, 0));
  if (NP == 4) {
    const __amdgpu_buffer_rsrc_t rJ = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(rows - shiftJ), (short)0, 0x7fffffff, 0x00020000);
    raw[2] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rJ, (int)offJ, 0, 0));
    raw[3] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rJ, (int)offJ, s16, 0));
  }
}

// General path (frame edges, unaligned rows, ragged tails): byte loads of the
// piece at time t, inputs n_first..n_first+15, delayed by d samples (row
// t - d, which may lie in the history before the frame); absent samples and
// inputs read as the code of 0 + 0i.
__device__ __forceinline__ v4i load_piece_edge(const uint8_t* __restrict__ samples,
                                               long long row_stride, int f, int N, int n_first,
                                               int t, int t_end, int d = 0) {
  uint32_t w[4] = {0x88888888u, 0x88888888u, 0x88888888u, 0x88888888u};
  if (t < t_end) {
    const uint8_t* p = samples + (long long)(t - d) * row_stride + (long long)f * N + n_first;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      if (n_first + e < N) {
        const uint32_t sh = 8 * (e & 3);
        w[e >> 2] = (w[e >> 2] & ~(0xFFu << sh)) | ((uint32_t)p[e] << sh);
      }
    }
  }
  return v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
}

// The pieces of a thread (NP as in load_pieces_fast) by the general path;
// t_chunk is the chunk's first time.
template <int NP>
__device__ __forceinline__ void load_pieces_edge(v4i (&raw)[4], const uint8_t* __restrict__ samples,
                                                 long long row_stride, int f, int N, int nI,
                                                 int nJ, const StageRole& sr, int t_chunk,
                                                 int t_end, int dI = 0, int dJ = 0) {
  raw[0] = load_piece_edge(samples, row_stride, f, N, nI, t_chunk + sr.rI, t_end, dI);
  raw[1] = load_piece_edge(samples, row_stride, f, N, nI, t_chunk + sr.rI + 16, t_end, dI);
  if (NP == 4) {
    raw[2] = load_piece_edge(samples, row_stride, f, N, nJ, t_chunk + sr.rJ, t_end, dJ);
    raw[3] = load_piece_edge(samples, row_stride, f, N, nJ, t_chunk + sr.rJ + 16, t_end, dJ);
  }
}

// Store a piece, unchanged, into the LDS plane of its block (rows = times, as
// loaded).  The nibbles are split after the transpose read (see
// compute_chunk).
//
// The operands are the offset-binary codes u = v + 8 in 0..15, which both
// matrix-core forms take as they are: as int8 they are the integers 0..15, and
// as FP8 e4m3 bytes they are u * 2^-9 (the subnormals 0..7 and the first
// binade 8..15 lie on one grid), which the MFMA's operand scale of 2^9 turns
// back into u.  The MFMA therefore integrates products of codes; the offsets
// are removed at the write from the per-input sums of the codes (see
// TileSums): with S_n = sum_t u_n,
//
//   sum (u_i - 8)(u_j - 8) = sum u_i u_j - 8 S_i - 8 S_j + 64 T.
__device__ __forceinline__ void stage_piece(const v4i& raw, uint8_t* __restrict__ dst) {
  *reinterpret_cast<v4i*>(dst) = raw;
}

// Piece k of a thread into the stage at `stage` (I block at 0, J block at
// BLOCK_LDS).
__device__ __forceinline__ void stage_piece_k(const v4i& raw, int k, uint8_t* __restrict__ stage,
                                              const StageRole& sr) {
  if (k < 2)
    stage_piece(raw, stage + (sr.rI + 16 * k) * PROW + 16 * sr.seg);
  else
    stage_piece(raw, stage + BLOCK_LDS + (sr.rJ + 16 * (k - 2)) * PROW + 16 * sr.seg);
}

template <int NP>
__device__ __forceinline__ void stage_pieces(const v4i (&raw)[4], uint8_t* __restrict__ stage,
                                             const StageRole& sr) {
#pragma unroll
  for (int k = 0; k < NP; ++k) stage_piece_k(raw[k], k, stage, sr);
}

template <int FORM>
struct Acc;
template <>
struct Acc<FORM_I8> {
  typedef v16i T;
};
template <>
struct Acc<FORM_F8> {
  typedef v16f T;
};

// Per-lane sums of codes over a tile's samples: of the real (r) and imaginary
// (m) codes of one 32-input A fragment (rows) and one B fragment (columns).
// Lane l sums input l & 31 of its fragment over the half of every k-step's
// samples it holds (l >> 5 selects the half).  Every wave sums the A fragment
// SA and the B fragment SB it is assigned, so that the four waves cover the
// 128 rows and 128 columns of the tile once.
//
// The codes (0..15) are added bytewise, as packed words (one add of three
// operands per two words: no carry leaves a byte while a byte holds at most
// 17 codes), into b*.  flush() folds the four bytes of each and adds them to
// the thread's 32-bit sums, which live in LDS, in the otherwise unused
// padding of the first stage's plane rows (bytes 128..159 of every 160-byte
// row; see sum_slot), so that they cost no registers.  It runs at most every
// 16 codes per byte, i.e. every two chunks.
struct TileSums {
  uint32_t bar, bam, bbr, bbm;  // bytewise partial sums since the last flush
};

// This thread's four 32-bit sums (ar, am, br, bm): a 16-byte slot in the
// padding of plane row tid / 2 of the first stage (rows 0..127 of its I-block
// planes), bytes 128 + 16 (tid & 1) on.  Staging writes and transpose reads
// touch bytes 0..127 of a row only.
__device__ __forceinline__ uint32_t* sum_slot(uint8_t* lds) {
  const int tid = threadIdx.x;
  return reinterpret_cast<uint32_t*>(lds + (tid >> 1) * PROW + BT + 16 * (tid & 1));
}

__device__ __forceinline__ void flush_sums(TileSums& sm, uint8_t* lds) {
  uint32_t* p = sum_slot(lds);
  atomicAdd(p + 0, __builtin_amdgcn_udot4(sm.bar, 0x01010101u, 0u, false));
  atomicAdd(p + 1, __builtin_amdgcn_udot4(sm.bam, 0x01010101u, 0u, false));
  atomicAdd(p + 2, __builtin_amdgcn_udot4(sm.bbr, 0x01010101u, 0u, false));
  atomicAdd(p + 3, __builtin_amdgcn_udot4(sm.bbm, 0x01010101u, 0u, false));
  sm.bar = sm.bam = sm.bbr = sm.bbm = 0u;
}

// Two words of codes added bytewise into acc.
__device__ __forceinline__ uint32_t badd(int x, int y, uint32_t acc) {
  return acc + (uint32_t)x + (uint32_t)y;
}

// FP8 operand scale: e8m0 exponent 127 + 9, i.e. 2^9 (code u reads u * 2^-9).
constexpr int F8_SCALE = 127 + 9;

// What one wave does in a tile's chunk loop.  Every field is a compile-time
// constant, so that the loops stay straight-line code.
//   SA, SB  the A and B fragment (0 or 1) whose codes the wave sums (-1: none)
//   KPAR    the k-steps it computes: 0 all; 1 the even and 2 the odd ones (two
//           waves share one 64 x 64 sub-tile of a diagonal tile)
//   SKIP10  no MFMAs for block (a = 1, b = 0), which lies below the diagonal
//           in a sub-tile on the diagonal
//   DIAG    a diagonal tile (I == J): only the I block is staged, and the B
//           fragments are read from it too
//   COMPUTE issue MFMAs (false: a wave whose sub-tile lies below the diagonal
//           only sums its fragments)
template <int SA_, int SB_, int KPAR_, bool SKIP10_, bool DIAG_, bool COMPUTE_ = true>
struct Role {
  static constexpr int SA = SA_, SB = SB_, KPAR = KPAR_;
  static constexpr bool SKIP10 = SKIP10_, DIAG = DIAG_, COMPUTE = COMPUTE_;
  static constexpr bool SUMS = SA_ >= 0 || SB_ >= 0;
  static constexpr int NP = DIAG_ ? 2 : 4;  // pieces a thread loads and stages per chunk
};

// One chunk for a wave's 64 x 64 sub-tile (2 x 2 blocks of 32 x 32).
// lds: the chunk's stage (I block at 0, J block at BLOCK_LDS); lane_rd: this
// lane's transpose-read offset within a k-step (its row group and column);
// rowA / rowB: the wave's first input row within the I and J blocks.
//
// R: the wave's role (see Role).  STAGE: the pieces `stg` of the next chunk
// are staged into the stage at `blk` between the k-steps (spread evenly over
// them), so that the staging issues while the matrix cores work.
//
// Operands.  Int8: a lane's 16 bytes pack [m(8), r(8)] for 8 samples; Re =
// A.B and Im = A.Y with Y = [r(8), 15 - m(8)] (15 - m = m ^ 15 per byte, one
// operation; the extra 15 sum_t r_i is removed with the sums).  Every int8
// operand byte thus lies in 0..15: small non-negative operands cost the
// matrix cores markedly less power than signed ones, and the kernel runs at
// the power limit.  Y is B's registers shifted by two, with 15 - m appended.
// FP8: a lane's 32 bytes pack [r(8), m(8), r(8), m(8)] for 16 samples; Y =
// [-m, r, -m, r], the negation flipping the sign bit.
template <int FORM, class R, bool STAGE>
__device__ __forceinline__ void compute_chunk(const uint8_t* __restrict__ lds, int lane_rd,
                                              int rowA, int rowB,
                                              typename Acc<FORM>::T (&re)[2][2],
                                              typename Acc<FORM>::T (&im)[2][2], TileSums& sm,
                                              const v4i* stg = nullptr, uint8_t* blk = nullptr,
                                              const StageRole* sr = nullptr) {
  const uint8_t* pa = lds + lane_rd + rowA;
  const uint8_t* pb = lds + (R::DIAG ? 0 : BLOCK_LDS) + lane_rd + rowB;
  if (FORM == FORM_I8) {
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      const bool kon = R::COMPUTE && (R::KPAR == 0 || (s & 1) == R::KPAR - 1);
      v4i A[2], B[2], Y[2];
      v2i ar[2], am[2], br[2], bm[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (!kon && a != R::SA) continue;
        const v2i w = lds_tr8(pa + 16 * s * PROW + 32 * a);
        ar[a] = hi_codes(w);
        am[a] = lo_codes(w);
        A[a] = v4i{am[a].x, am[a].y, ar[a].x, ar[a].y};
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (!kon && b != R::SB) continue;
        const v2i wb = lds_tr8(pb + 16 * s * PROW + 32 * b);
        br[b] = hi_codes(wb);
        bm[b] = lo_codes(wb);
        const int c15 = 0x0F0F0F0F;
        const v8i w = v8i{bm[b].x, bm[b].y, br[b].x, br[b].y, bm[b].x ^ c15, bm[b].y ^ c15, 0, 0};
        B[b] = __builtin_shufflevector(w, w, 0, 1, 2, 3);
        Y[b] = __builtin_shufflevector(w, w, 2, 3, 4, 5);
      }
      if (kon) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            if (R::SKIP10 && a == 1 && b == 0) continue;
            re[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], B[b], re[a][b], 0, 0, 0);
            im[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], Y[b], im[a][b], 0, 0, 0);
          }
      }
      if constexpr (R::SA >= 0) {
        sm.bar = badd(ar[R::SA].x, ar[R::SA].y, sm.bar);
        sm.bam = badd(am[R::SA].x, am[R::SA].y, sm.bam);
      }
      if constexpr (R::SB >= 0) {
        sm.bbr = badd(br[R::SB].x, br[R::SB].y, sm.bbr);
        sm.bbm = badd(bm[R::SB].x, bm[R::SB].y, sm.bbm);
      }
      if (STAGE) {
        if (R::NP == 4)
          stage_piece_k(stg[s], s, blk, *sr);
        else if ((s & 1) == 0)
          stage_piece_k(stg[s >> 1], s >> 1, blk, *sr);
      }
    }
  } else {
    // a lane's 32 operand bytes: two groups of 8 samples (rows +0..7, +8..15)
#pragma unroll
    for (int s = 0; s < KC / 32; ++s) {
      const bool kon = R::COMPUTE && (R::KPAR == 0 || s == R::KPAR - 1);
      v8i A[2], B[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (!kon && a != R::SA) continue;
        const uint8_t* q = pa + 32 * s * PROW + 32 * a;
        const v2i w0 = lds_tr8(q), w1 = lds_tr8(q + 8 * PROW);
        const v2i r0 = hi_codes(w0), m0 = lo_codes(w0), r1 = hi_codes(w1), m1 = lo_codes(w1);
        A[a] = v8i{r0.x, r0.y, m0.x, m0.y, r1.x, r1.y, m1.x, m1.y};
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (!kon && b != R::SB) continue;
        const uint8_t* q = pb + 32 * s * PROW + 32 * b;
        const v2i w0 = lds_tr8(q), w1 = lds_tr8(q + 8 * PROW);
        const v2i r0 = hi_codes(w0), m0 = lo_codes(w0), r1 = hi_codes(w1), m1 = lo_codes(w1);
        B[b] = v8i{r0.x, r0.y, m0.x, m0.y, r1.x, r1.y, m1.x, m1.y};
      }
      if (kon) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // FP8 negation flips the sign bit: [r r m m] -> [-m -m r r]
          const int sg = (int)0x80808080u;
          const v8i Y = v8i{B[b][2] ^ sg, B[b][3] ^ sg, B[b][0], B[b][1],
                            B[b][6] ^ sg, B[b][7] ^ sg, B[b][4], B[b][5]};
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            if (R::SKIP10 && a == 1 && b == 0) continue;
            // format 0 = FP8 e4m3 for both operands; both scales 2^9
            re[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                A[a], B[b], re[a][b], 0, 0, 0, F8_SCALE, 0, F8_SCALE);
            im[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                A[a], Y, im[a][b], 0, 0, 0, F8_SCALE, 0, F8_SCALE);
          }
        }
      }
      if constexpr (R::SA >= 0) {
        const v8i sA = A[R::SA];
        sm.bar = badd(sA[4], sA[5], badd(sA[0], sA[1], sm.bar));
        sm.bam = badd(sA[6], sA[7], badd(sA[2], sA[3], sm.bam));
      }
      if constexpr (R::SB >= 0) {
        const v8i sB = B[R::SB];
        sm.bbr = badd(sB[4], sB[5], badd(sB[0], sB[1], sm.bbr));
        sm.bbm = badd(sB[6], sB[7], badd(sB[2], sB[3], sm.bbm));
      }
      if (STAGE) {
        if (R::NP == 4) {
          stage_piece_k(stg[2 * s], 2 * s, blk, *sr);
          stage_piece_k(stg[2 * s + 1], 2 * s + 1, blk, *sr);
        } else {
          stage_piece_k(stg[s], s, blk, *sr);
        }
      }
    }
  }
}

// This lane's transpose-read offset within a k-step: lanes of a 16-lane group
// g address rows (j >> 1) at columns 8 * (j & 1) of a 16-input half; groups
// 0/1 hold inputs 0..15 / 16..31 of a 32-row fragment, groups 2/3 the same
// inputs eight (int8) or sixteen (FP8) samples later.
template <int FORM>
__device__ __forceinline__ int lane_read_offset(int lane) {
  const int g = lane >> 4, j = lane & 15;
  const int row = (FORM == FORM_I8 ? 8 : 16) * (g >> 1) + (j >> 1);
  return row * PROW + 16 * (g & 1) + 8 * (j & 1);
}

// Accumulator values as 32-bit words and back (by value: an element of a
// vector register is not an object whose bytes can be reinterpreted).
__device__ __forceinline__ uint32_t acc_bits(int x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t acc_bits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ int acc_from_bits(uint32_t b, int) { return (int)b; }
__device__ __forceinline__ float acc_from_bits(uint32_t b, float) { return __uint_as_float(b); }

__device__ __forceinline__ int to_i32(int x) { return x; }
__device__ __forceinline__ int to_i32(float x) { return (int)x; }  // exact: integral, |x| < 2^24

// Offset corrections of one input, added at the write (see stage_piece):
// with S_r, S_m the sums of its real and imaginary codes over the T samples a
// tile integrated (padding included: padded samples are codes 8 + 8i),
//
//   Re V_ij = Re_ij - 8 (S_r,i + S_m,i + S_r,j + S_m,j) + 128 T
//   Im V_ij = Im_ij - 8 (S_m,i - S_r,i) + 8 (S_m,j - S_r,j)   [- 15 S_r,i for
//             int8, whose Y carries 15 - m instead of -m].
// Row terms (A side) carry the constant 128 T.
struct Corr {
  int re, im;
};

template <int FORM>
__device__ __forceinline__ Corr row_corr(int sr, int sm, int T) {
  return Corr{128 * T - 8 * (sr + sm), 8 * (sr - sm) - (FORM == FORM_I8 ? 15 * sr : 0)};
}
__device__ __forceinline__ Corr col_corr(int sr, int sm) {
  return Corr{-8 * (sr + sm), 8 * (sm - sr)};
}

// K baselines of one lane into vis: (vr[v], vi[v]) into pair b[v] of base
// (b(i, j) = i N - i (i - 1) / 2 + (j - i)), for the v set in ok, in write
// mode MODE.
//
// WM_ATOMIC64: the pair (re, im), read as the 64-bit integer
// re + 2^32 (im + [re < 0]), takes one atomic add of vr + 2^32 vi, which is
// exact; the add moves a borrow between the words exactly when the sign of
// the real word changes (the returned old value tells), and a 32-bit add on
// the imaginary word takes it back.  Once every add of a launch has landed,
// the pair is (sum re, sum im) again, so that work items adding into one
// baseline cost one wide atomic each instead of two.  All K wide adds issue
// before the first returned value is needed.
template <int MODE, int K>
__device__ __forceinline__ void put_pairs(int32_t* base, const int (&b)[K], const int (&vr)[K],
                                          const int (&vi)[K], uint32_t ok) {
  if constexpr (MODE == WM_ATOMIC64) {
    uint32_t old[K];
#pragma unroll
    for (int v = 0; v < K; ++v) {
      old[v] = 0u;
      if (ok & (1u << v)) {
        const unsigned long long add =
            ((unsigned long long)(uint32_t)vi[v] << 32) + (unsigned long long)(long long)vr[v];
        old[v] = (uint32_t)atomicAdd(reinterpret_cast<unsigned long long*>(base + 2 * b[v]), add);
      }
    }
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const int re0 = (int)old[v];
      const int re1 = (int)(old[v] + (uint32_t)vr[v]);
      const int fix = (re1 < 0) - (re0 < 0);
      if ((ok & (1u << v)) && fix) atomicAdd(base + 2 * b[v] + 1, fix);
    }
  } else {
#pragma unroll
    for (int v = 0; v < K; ++v) {
      if (!(ok & (1u << v))) continue;
      int32_t* p = base + 2 * b[v];
      if constexpr (MODE == WM_STORE) {
        *reinterpret_cast<int2*>(p) = make_int2(vr[v], vi[v]);
      } else if constexpr (MODE == WM_ADD) {
        const int2 q = *reinterpret_cast<int2*>(p);
        *reinterpret_cast<int2*>(p) = make_int2(q.x + vr[v], q.y + vi[v]);
      } else {
        atomicAdd(p, vr[v]);
        if (vi[v]) atomicAdd(p + 1, vi[v]);
      }
    }
  }
}

// The mode a work item writes in: its int32 atomic adds become one 64-bit
// atomic per baseline where vis is 8-byte aligned (every channel's and gate's
// triangle then is).
__device__ __forceinline__ int wide_atomics(int mode, const int32_t* vis) {
  return mode == WM_ATOMIC && !(reinterpret_cast<uintptr_t>(vis) & 7) ? (int)WM_ATOMIC64 : mode;
}

// Packed index of baseline (i, j), i <= j (unsigned arithmetic: callers also
// form it for rows past N, whose index they never use).
__device__ __forceinline__ int pair_index(int i, int j, int N) {
  return (int)((uint32_t)i * (uint32_t)N - (((uint32_t)i * (uint32_t)(i - 1)) >> 1) +
               (uint32_t)(j - i));
}

// Write a wave's finished blocks into the packed triangle, adding the offset
// corrections (corr: 128 row terms, then 128 column terms, in LDS).  Offsets
// within a channel are 32-bit (the plan limits N so that 2 N(N+1)/2 < 2^31).
template <int MODE, class V>
__device__ __forceinline__ void write_blocks_m(int32_t* base, int N, int rs0, int cs0, int lr0,
                                               int lc0, const int2* corr, int lane, int mask,
                                               V (&re)[2][2], V (&im)[2][2]) {
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int ai = ab >> 1, bi = ab & 1;
    if (!(mask & (1 << ab))) continue;
    const int j = cs0 + 32 * bi + (lane & 31);
    const int2 cj = corr[128 + lc0 + 32 * bi + (lane & 31)];
    // two groups of eight registers (fewer live values beside the
    // accumulators still to be written)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int b[8], vr[8], vi[8];
      uint32_t ok = 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int v = 8 * h + u;
        const int di = 32 * ai + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int i = rs0 + di;
        const int2 ci = corr[lr0 + di];
        ok |= (uint32_t)(i < N && j < N && j >= i) << u;
        b[u] = pair_index(i, j, N);
        vr[u] = to_i32(re[ai][bi][v]) + ci.x + cj.x;
        vi[u] = (i == j) ? 0 : to_i32(im[ai][bi][v]) + ci.y + cj.y;
      }
      put_pairs<MODE>(base, b, vr, vi, ok);
    }
  }
}

// WIDE: 32-bit atomic adds become 64-bit ones where vis allows (see
// put_pairs).  Only the kernels that take it: the wide path's registers
// change how the compiler lays out the plain kernel's chunk loop (measured
// slower there), while the persistent kernel, whose tiles are often split in
// time, gains.
template <bool WIDE, class V>
__device__ __forceinline__ void write_blocks(int32_t* vis, int N, long long NB, int f, int rs0,
                                             int cs0, int lr0, int lc0, const int2* corr,
                                             int lane, int mask, int mode, V (&re)[2][2],
                                             V (&im)[2][2]) {
  int32_t* base = vis + 2 * (long long)f * NB;
  if (WIDE && wide_atomics(mode, vis) == WM_ATOMIC64) {
    write_blocks_m<WM_ATOMIC64>(base, N, rs0, cs0, lr0, lc0, corr, lane, mask, re, im);
    return;
  }
  // stores, read-add-stores and 32-bit atomics one baseline at a time (the
  // fewest live registers: the chunk loop keeps its allocation)
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int ai = ab >> 1, bi = ab & 1;
    if (!(mask & (1 << ab))) continue;
    const int j = cs0 + 32 * bi + (lane & 31);
    const int2 cj = corr[128 + lc0 + 32 * bi + (lane & 31)];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int di = 32 * ai + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      const int i = rs0 + di;
      if (i < N && j < N && j >= i) {
        const int2 ci = corr[lr0 + di];
        int32_t* p = base + 2 * pair_index(i, j, N);
        const int vr = to_i32(re[ai][bi][v]) + ci.x + cj.x;
        const int vi = (i == j) ? 0 : to_i32(im[ai][bi][v]) + ci.y + cj.y;
        if (mode == WM_STORE) {
          *reinterpret_cast<int2*>(p) = make_int2(vr, vi);
        } else if (mode == WM_ADD) {
          int2 o = *reinterpret_cast<int2*>(p);
          *reinterpret_cast<int2*>(p) = make_int2(o.x + vr, o.y + vi);
        } else {
          atomicAdd(p, vr);
          if (vi) atomicAdd(p + 1, vi);
        }
      }
    }
  }
}

// Row-major upper-triangle tile index p -> (I, J), I <= J < nt.
__device__ __forceinline__ void tile_of(int p, int nt, int& I, int& J) {
  const float w = 2.0f * nt + 1.0f;
  int i = (int)((w - __builtin_sqrtf(w * w - 8.0f * p)) * 0.5f);
  if (i < 0) i = 0;
  if (i > nt - 1) i = nt - 1;
  // correct the float estimate: start(i) = i*nt - i(i-1)/2
  while (i > 0 && i * nt - i * (i - 1) / 2 > p) --i;
  while (i + 1 < nt && (i + 1) * nt - (i + 1) * i / 2 <= p) ++i;
  I = i;
  J = i + (p - (i * nt - i * (i - 1) / 2));
}

// Everything one thread needs to stage and compute chunks of a tile.
template <int FORM>
struct TileCtx {
  uint8_t* lds;
  const uint8_t* rows;  // channel's rows at the tile's first sample (uniform)
  long long row_stride;
  uint32_t offI, offJ;  // this thread's loads: its first I / J row and its inputs
  long long shiftI, shiftJ;  // time shifting: block delays in bytes (uniform)
  int dI, dJ;                // time shifting: this thread's segment delays (rows)
  StageRole sr;
  int lane_rd, rowA, rowB;
  typename Acc<FORM>::T re[2][2], im[2][2];
  TileSums sm;
  __device__ __forceinline__ explicit TileCtx(int h) : sr(h) {}
};

// One chunk of the steady state: optionally load chunk `ld_chunk` into `ld`,
// compute the chunk staged at `cur` while staging `stg` into `nxt`, then
// synchronise.  Straight-line code, so that the compiler can interleave the
// staging arithmetic with the matrix instructions.
template <int FORM, class R>
__device__ __forceinline__ void steady_step(TileCtx<FORM>& x, int cur, int nxt, const v4i (&stg)[4],
                                            v4i (&ld)[4], int ld_chunk) {
  load_pieces_fast<R::NP>(ld, x.rows + (long long)ld_chunk * KC * x.row_stride, x.row_stride,
                          x.offI, x.offJ, x.shiftI, x.shiftJ);
  // keep the loads at the top of the step: they have a whole step to land
  __builtin_amdgcn_sched_barrier(0);
  compute_chunk<FORM, R, true>(x.lds + cur, x.lane_rd, x.rowA, x.rowB, x.re, x.im, x.sm, stg,
                               x.lds + nxt, &x.sr);
  __syncthreads();
}

// Chunks [0, nsteady) of a tile, nsteady even and >= 2, all of whose loads
// lie inside the frame (chunks < nfast).  Chunk c computes from buffer c & 1
// while chunk c + 1 is staged into the other buffer and chunk c + 2 loads
// (two register sets of raw samples).  Prefetches past the last fast chunk
// reload that chunk, and what they stage is never computed, so the loop body
// has no branch.
template <int FORM, class R>
__device__ __forceinline__ void steady_chunks(TileCtx<FORM>& x, int nsteady, int nfast) {
  constexpr int B0 = 0, B1 = STAGE_LDS;
  v4i rawA[4], rawB[4];
  load_pieces_fast<R::NP>(rawA, x.rows, x.row_stride, x.offI, x.offJ, x.shiftI, x.shiftJ);
  stage_pieces<R::NP>(rawA, x.lds + B0, x.sr);
  load_pieces_fast<R::NP>(rawA, x.rows + (long long)KC * x.row_stride, x.row_stride, x.offI,
                          x.offJ, x.shiftI, x.shiftJ);
  __syncthreads();
  for (int c = 0; c < nsteady; c += 2) {
    steady_step<FORM, R>(x, B0, B1, rawA, rawB, min(c + 2, nfast - 1));
    steady_step<FORM, R>(x, B1, B0, rawB, rawA, min(c + 3, nfast - 1));
    // two chunks: 8 x 2 (int8) or 4 x 4 (FP8) words, <= 240 a byte
    if (R::SUMS) flush_sums(x.sm, x.lds);
  }
}

// The same with one register set: chunk c + 1 loads at the start of chunk
// c's step and is staged after chunk c's MFMAs.  Sixteen fewer registers:
// for the FP8 form (wider operands) and shifted frames.
template <int FORM, class R>
__device__ __forceinline__ void steady_step1(TileCtx<FORM>& x, int cur, int nxt, v4i (&raw)[4],
                                             int ld_chunk) {
  load_pieces_fast<R::NP>(raw, x.rows + (long long)ld_chunk * KC * x.row_stride, x.row_stride,
                          x.offI, x.offJ, x.shiftI, x.shiftJ);
  __builtin_amdgcn_sched_barrier(0);
  compute_chunk<FORM, R, false>(x.lds + cur, x.lane_rd, x.rowA, x.rowB, x.re, x.im, x.sm);
  __builtin_amdgcn_sched_barrier(0);
  stage_pieces<R::NP>(raw, x.lds + nxt, x.sr);
  __syncthreads();
}

template <int FORM, class R>
__device__ __forceinline__ void steady_chunks1(TileCtx<FORM>& x, int nsteady, int nfast) {
  constexpr int B0 = 0, B1 = STAGE_LDS;
  v4i raw[4];
  load_pieces_fast<R::NP>(raw, x.rows, x.row_stride, x.offI, x.offJ, x.shiftI, x.shiftJ);
  stage_pieces<R::NP>(raw, x.lds + B0, x.sr);
  __syncthreads();
  for (int c = 0; c < nsteady; c += 2) {
    steady_step1<FORM, R>(x, B0, B1, raw, min(c + 1, nfast - 1));
    steady_step1<FORM, R>(x, B1, B0, raw, min(c + 2, nfast - 1));
    if (R::SUMS) flush_sums(x.sm, x.lds);
  }
}

template <int FORM, bool DEEP, class R>
__device__ __forceinline__ void steady(TileCtx<FORM>& x, int nsteady, int nfast) {
  if (DEEP)
    steady_chunks<FORM, R>(x, nsteady, nfast);
  else
    steady_chunks1<FORM, R>(x, nsteady, nfast);
}

// Time ranges a tile integrates: one range [t0, t1) ...
struct OneRange {
  static constexpr bool kSingle = true;
  int t0, t1;
  __device__ __forceinline__ int count() const { return 1; }
  __device__ __forceinline__ int begin(int) const { return t0; }
  __device__ __forceinline__ int end(int) const { return t1; }
};

// ... or a list of runs [x, y) (output gating: the runs of one gate).
struct RunList {
  static constexpr bool kSingle = false;
  const int2* runs;
  int n;
  __device__ __forceinline__ int count() const { return n; }
  __device__ __forceinline__ int begin(int r) const { return runs[r].x; }
  __device__ __forceinline__ int end(int r) const { return runs[r].y; }
};

// The chunks of one time range [t_begin, t_end) of a tile, added into the
// tile's accumulators and sums.  Returns the samples it integrated, padding
// of a ragged last chunk included (padded samples are the code 8 + 8i).
// R: the wave's role (see Role; fixed per wave, see tile_body).
template <int FORM, bool ALIGNED, bool DEEP, class R>
__device__ __forceinline__ int tile_range(TileCtx<FORM>& x, const uint8_t* __restrict__ samples,
                                          int N, int f, int nI, int nJ, int t_begin, int t_end,
                                          uint8_t* lds) {
  const int len = t_end > t_begin ? t_end - t_begin : 0;
  const int nchunks = (len + KC - 1) / KC;
  const long long row_stride = x.row_stride;
  // uniform row pointer of this channel at t_begin
  const uint8_t* rows = samples + (long long)t_begin * row_stride + (long long)f * N;
  x.rows = rows;

  // Steady state over the chunks whose loads all lie inside the frame.
  const int nfast = ALIGNED ? len / KC : 0;
  const int nsteady = nfast & ~1;
  int c = 0;
  if (nsteady >= 2) {
    steady<FORM, DEEP, R>(x, nsteady, nfast);
    c = nsteady;
  }

  // General loop: the remaining chunks (frame edges, ragged tail, short
  // ranges), one buffer flip per chunk.
  v4i raw[4];
  auto load = [&](int cc) {
    if (ALIGNED && (cc + 1) * KC <= len)
      load_pieces_fast<R::NP>(raw, rows + (long long)cc * KC * row_stride, row_stride, x.offI,
                              x.offJ, x.shiftI, x.shiftJ);
    else
      load_pieces_edge<R::NP>(raw, samples, row_stride, f, N, nI, nJ, x.sr, t_begin + cc * KC,
                              t_end, x.dI, x.dJ);
  };
  if (c < nchunks) {
    load(c);
    stage_pieces<R::NP>(raw, lds + (c & 1) * STAGE_LDS, x.sr);
    __syncthreads();
  }
  for (; c < nchunks; ++c) {
    uint8_t* cur = lds + (c & 1) * STAGE_LDS;
    uint8_t* nxt = lds + ((c + 1) & 1) * STAGE_LDS;
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    compute_chunk<FORM, R, false>(cur, x.lane_rd, x.rowA, x.rowB, x.re, x.im, x.sm);
    if (R::SUMS) flush_sums(x.sm, lds);
    if (more) stage_pieces<R::NP>(raw, nxt, x.sr);
    __syncthreads();
  }
  return nchunks * KC;
}

// All ranges of a tile for one wave role.
template <int FORM, bool ALIGNED, bool DEEP, class R, class Ranges>
__device__ __forceinline__ int tile_ranges(TileCtx<FORM>& x, const uint8_t* __restrict__ samples,
                                           int N, int f, int nI, int nJ, const Ranges& rg,
                                           uint8_t* lds) {
  if constexpr (Ranges::kSingle) {
    return tile_range<FORM, ALIGNED, DEEP, R>(x, samples, N, f, nI, nJ, rg.begin(0), rg.end(0),
                                              lds);
  } else {
    int teff = 0;
    for (int r = 0; r < rg.count(); ++r)
      teff += tile_range<FORM, ALIGNED, DEEP, R>(x, samples, N, f, nI, nJ, rg.begin(r),
                                                 rg.end(r), lds);
    return teff;
  }
}

// LDS of a tile's epilogue, once its chunks are done: the per-input partial
// sums (part[half][side][plane][128]) and the offset corrections (corr: 128
// row terms, then 128 column terms) at the end of the LDS, clear of the
// first 32 KiB, through which the two waves that share a sub-tile of a
// diagonal tile exchange accumulators.
constexpr int EPI_PART = LDS_BYTES - 2 * 2 * 2 * BT * 4 - 2 * BT * 8;
constexpr int EPI_CORR = LDS_BYTES - 2 * BT * 8;
constexpr int EPI_SWAP = 64 * 64 * 4;  // bytes one wave hands over: 64 values a lane
static_assert(2 * EPI_SWAP <= EPI_PART, "epilogue regions overlap");

// The work of one tile: baselines [I*128, I*128+128) x [J*128, J*128+128) of
// channel f, integrated over the time ranges `rg`.  All 256 threads call it;
// it ends with the tile written (mode) and the LDS free for reuse.
// FP8 form: the caller keeps the integrated samples <= XENG_F8_FLUSH_MAX, so
// that every f32 partial sum of codes is an integer below 2 * 225 * 32768 <
// 2^24 (exact).  Int8 form: the caller keeps them <= XENG_I8_SEG_MAX, so that
// the int32 sums of codes stay below 2 * 225 * 2^19 < 2^31.
//
// ALIGNED: N % 16 == 0 and the sample rows are 16-byte aligned, so that whole
// chunks can take the fast loads.  DEEP: prefetch two chunks ahead (else one).
//
// Wave roles.  Off the diagonal (I < J), wave (wr, wc) computes the 64 x 64
// sub-tile (wr, wc) and sums A fragment wc and B fragment wr, so that the
// four waves cover the tile's 128 rows and 128 columns once.  On the diagonal
// (I == J) sub-tile (1, 0) lies below the diagonal.  Without SPLITDIAG the
// waves keep their roles there, and wave 2 only sums its fragments.  With
// SPLITDIAG (fewer MFMAs and half the staging in a diagonal tile, for frames
// with a large share of diagonal tiles), waves 0 and 3 compute the
// diagonal sub-tiles (0, 0) and (1, 1), skipping their block below the
// diagonal, and sum the 64 inputs of their sub-tile (rows and columns are the
// same inputs); waves 1 and 2 share sub-tile (0, 1), wave 1 taking the even
// and wave 2 the odd k-steps, and at the end each hands the other the half of
// the sub-tile it does not write.  Only the I block is staged there.  A wave
// whose blocks all lie past N computes anyway (its results are never
// written), so that every role has one instantiation.  The role is a
// compile-time parameter of the chunk loops, dispatched once per tile on the
// wave index.
//
// Time shifting (Sec. IV-C, "Time Shifting"): with seg_delay (delays per
// 16-input segment, in samples) and blk_delay (their maximum per 128-input
// block), input n is read at time t - delay(n); rows before the frame come
// from the history the caller keeps in front of `samples`.  A block's largest
// delay moves its (scalar) load base back; a lane's offset adds back the rows
// its own segment is delayed less.  NULL tables: no shift.
template <int FORM, bool ALIGNED, bool DEEP, bool SHIFT, class Ranges, bool SPLITDIAG = true,
          bool WIDE = false>
__device__ __forceinline__ void tile_body(const uint8_t* __restrict__ samples, int32_t* vis,
                                          int N, long long row_stride, long long NB, int f,
                                          int I, int J, const Ranges& rg, int mode,
                                          uint8_t* lds, const int* seg_delay = nullptr,
                                          const int* blk_delay = nullptr) {
  // the wave index is uniform per wave: read it into a scalar register so that
  // every branch on it is a uniform one.  The thread index passes through an
  // empty asm statement, so that what the tile derives from it is computed
  // per tile: the persistent kernel would otherwise keep those values live
  // (and spilled) across its whole loop over tiles.
  int tid_opaque = threadIdx.x;
  asm volatile("" : "+v"(tid_opaque));
  const int tid = tid_opaque, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool diag = SPLITDIAG && I == J;  // the split roles of a diagonal tile
  const bool shared = diag && (wave == 1 || wave == 2);  // the shared sub-tile (0, 1)
  const int wr = shared ? 0 : wave >> 1, wc = shared ? 1 : wave & 1;

  // MFMA blocks of this wave's sub-tile that hold baselines of the triangle
  // (and, for the shared sub-tile, the half this wave writes)
  const int rs0 = I * BT + 64 * wr, cs0 = J * BT + 64 * wc;
  int mask = 0;
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int rs = rs0 + 32 * (ab >> 1), cs = cs0 + 32 * (ab & 1);
    if (rs < N && cs < N && cs >= rs) mask |= 1 << ab;
  }
  if (shared) mask &= wave == 1 ? 0x3 : 0xC;

  // staging role: every thread stages two I pieces and, off the diagonal,
  // two J pieces
  TileCtx<FORM> x(tid);
  const int nI = I * BT + 16 * x.sr.seg, nJ = J * BT + 16 * x.sr.seg;
  // the lane's load offsets; fast loads of inputs past N (edge tiles,
  // N % 16 == 0) read a valid row instead: their LDS rows only reach
  // baselines past N, never written
  x.lds = lds;
  x.row_stride = row_stride;
  int DI = 0, DJ = 0;
  x.dI = x.dJ = 0;
  if (SHIFT) {
    DI = blk_delay[I];
    DJ = blk_delay[J];
    x.dI = nI < N ? seg_delay[nI >> 4] : DI;
    x.dJ = nJ < N ? seg_delay[nJ >> 4] : DJ;
  }
  x.shiftI = (long long)DI * row_stride;
  x.shiftJ = (long long)DJ * row_stride;
  x.offI = (uint32_t)(x.sr.rI + DI - x.dI) * (uint32_t)row_stride + (uint32_t)(nI < N ? nI : 0);
  x.offJ = (uint32_t)(x.sr.rJ + DJ - x.dJ) * (uint32_t)row_stride + (uint32_t)(nJ < N ? nJ : 0);
  x.lane_rd = lane_read_offset<FORM>(lane);
  x.rowA = 64 * wr;
  x.rowB = 64 * wc;
  x.sm = TileSums{0u, 0u, 0u, 0u};
  // clear this thread's sums slot (it alone adds to it; a wave's LDS
  // operations complete in order, and the previous tile ended on a barrier).
  // The zeros, too, are made per tile (kept across the persistent kernel's
  // loop, a zero vector would be spilled).
  int zero = 0;
  asm volatile("" : "+v"(zero));
  *reinterpret_cast<v4i*>(sum_slot(lds)) = v4i{zero, zero, zero, zero};
  typedef typename Acc<FORM>::T V;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      x.re[p][q] = V{};
      x.im[p][q] = V{};
    }

  // samples integrated, padding of ragged chunks included; one dispatch on
  // the wave's role per tile (a dispatch inside a loop over ranges, or a loop
  // around one, costs the compiler many registers)
  int teff;
#define XENG_RANGES(...) \
  tile_ranges<FORM, ALIGNED, DEEP, Role<__VA_ARGS__>>(x, samples, N, f, nI, nJ, rg, lds)
  if (diag) {
    switch (wave) {
      case 1: teff = XENG_RANGES(-1, -1, 1, false, true); break;
      case 2: teff = XENG_RANGES(-1, -1, 2, false, true); break;
      default: teff = XENG_RANGES(0, 1, 0, true, true); break;
    }
  } else {
    switch (wave) {
      case 0: teff = XENG_RANGES(0, 0, 0, false, false); break;
      case 1: teff = XENG_RANGES(1, 0, 0, false, false); break;
      case 2:
        if (!SPLITDIAG && I == J)  // below the diagonal: sums only
          teff = XENG_RANGES(0, 1, 0, false, false, false);
        else
          teff = XENG_RANGES(0, 1, 0, false, false);
        break;
      default: teff = XENG_RANGES(1, 1, 0, false, false); break;
    }
  }
#undef XENG_RANGES

  // Per-input sums -> offset corrections (see EPI_PART).  Off the diagonal a
  // lane of wave (wr, wc) holds rows 64 wr + 32 wc + l and columns
  // 64 wc + 32 wr + l; on the diagonal, waves 0 and 3 hold inputs 64 wr + l
  // (A fragment 0) and 64 wr + 32 + l (B fragment 1), and the column sums
  // are the row sums.
  if (!Ranges::kSingle && rg.count() == 0)
    __syncthreads();  // every sums slot is cleared before it is read
  int* part = reinterpret_cast<int*>(lds + EPI_PART);
  int2* corr = reinterpret_cast<int2*>(lds + EPI_CORR);
  {
    const v4i sums = *reinterpret_cast<const v4i*>(sum_slot(lds));
    const int h = lane >> 5, l = lane & 31;
    if (!diag) {
      const int ra = 64 * wr + 32 * wc + l, cb = 64 * wc + 32 * wr + l;
      part[((h * 2 + 0) * 2 + 0) * BT + ra] = sums.x;
      part[((h * 2 + 0) * 2 + 1) * BT + ra] = sums.y;
      part[((h * 2 + 1) * 2 + 0) * BT + cb] = sums.z;
      part[((h * 2 + 1) * 2 + 1) * BT + cb] = sums.w;
    } else if (!shared) {
      const int na = 64 * wr + l, nb = 64 * wr + 32 + l;
      part[((h * 2 + 0) * 2 + 0) * BT + na] = sums.x;
      part[((h * 2 + 0) * 2 + 1) * BT + na] = sums.y;
      part[((h * 2 + 0) * 2 + 0) * BT + nb] = sums.z;
      part[((h * 2 + 0) * 2 + 1) * BT + nb] = sums.w;
    }
  }
  __syncthreads();  // the partial sums are complete, and every sums slot has been read
  {
    const int side = tid >> 7, n = tid & (BT - 1);
    const int ps = diag ? 0 : side;
    const int sr = part[((0 * 2 + ps) * 2 + 0) * BT + n] + part[((1 * 2 + ps) * 2 + 0) * BT + n];
    const int sm = part[((0 * 2 + ps) * 2 + 1) * BT + n] + part[((1 * 2 + ps) * 2 + 1) * BT + n];
    const Corr cr = side == 0 ? row_corr<FORM>(sr, sm, teff) : col_corr(sr, sm);
    corr[side * BT + n] = make_int2(cr.re, cr.im);
  }
  // the shared sub-tile: wave 1 writes block row 0 and hands over its block
  // row 1, wave 2 the reverse (lane-minor, so that the exchange is free of
  // bank conflicts)
  uint32_t* swap = reinterpret_cast<uint32_t*>(lds);
  if (shared) {
    uint32_t* give = swap + (wave == 1 ? 0 : EPI_SWAP / 4);
    if (wave == 1) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          give[((0 * 2 + b) * 16 + v) * 64 + lane] = acc_bits(x.re[1][b][v]);
          give[((1 * 2 + b) * 16 + v) * 64 + lane] = acc_bits(x.im[1][b][v]);
        }
    } else {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          give[((0 * 2 + b) * 16 + v) * 64 + lane] = acc_bits(x.re[0][b][v]);
          give[((1 * 2 + b) * 16 + v) * 64 + lane] = acc_bits(x.im[0][b][v]);
        }
    }
  }
  __syncthreads();
  if (shared) {
    typedef typename std::remove_reference<decltype(x.re[0][0][0])>::type E;
    const uint32_t* take = swap + (wave == 1 ? EPI_SWAP / 4 : 0);
    if (wave == 1) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          x.re[0][b][v] += acc_from_bits(take[((0 * 2 + b) * 16 + v) * 64 + lane], E{});
          x.im[0][b][v] += acc_from_bits(take[((1 * 2 + b) * 16 + v) * 64 + lane], E{});
        }
    } else {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          x.re[1][b][v] += acc_from_bits(take[((0 * 2 + b) * 16 + v) * 64 + lane], E{});
          x.im[1][b][v] += acc_from_bits(take[((1 * 2 + b) * 16 + v) * 64 + lane], E{});
        }
    }
  }
  if (mask)
    write_blocks<WIDE>(vis, N, NB, f, rs0, cs0, 64 * wr, 64 * wc, corr, lane, mask, mode, x.re,
                       x.im);
  __syncthreads();  // the corrections are read before the LDS is reused
}

// Launch K<FORM, ALIGNED, SHIFT> for the run-time form, alignment and shift.
#define XENG_DISPATCH3(K, form, aligned, shift, g, b, stream, arg)                            \
  do {                                                                                        \
    if ((form) == FORM_I8) {                                                                  \
      if (aligned) {                                                                          \
        if (shift) hipLaunchKernelGGL((K<FORM_I8, true, true>), g, b, 0, stream, arg);        \
        else hipLaunchKernelGGL((K<FORM_I8, true, false>), g, b, 0, stream, arg);             \
      } else {                                                                                \
        if (shift) hipLaunchKernelGGL((K<FORM_I8, false, true>), g, b, 0, stream, arg);       \
        else hipLaunchKernelGGL((K<FORM_I8, false, false>), g, b, 0, stream, arg);            \
      }                                                                                       \
    } else {                                                                                  \
      if (aligned) {                                                                          \
        if (shift) hipLaunchKernelGGL((K<FORM_F8, true, true>), g, b, 0, stream, arg);        \
        else hipLaunchKernelGGL((K<FORM_F8, true, false>), g, b, 0, stream, arg);             \
      } else {                                                                                \
        if (shift) hipLaunchKernelGGL((K<FORM_F8, false, true>), g, b, 0, stream, arg);       \
        else hipLaunchKernelGGL((K<FORM_F8, false, false>), g, b, 0, stream, arg);            \
      }                                                                                       \
    }                                                                                         \
  } while (0)

}  // namespace xeng
