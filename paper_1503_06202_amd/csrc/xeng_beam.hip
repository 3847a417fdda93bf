// Discrete beamforming (Sec. IV-C, "Discrete Beamforming"): the data of all
// inputs are phase-shifted and summed so that a signal from one direction adds
// in phase, and the sum is written out at the sample cadence:
//
//     y[t][f][b] = sum_n w[f][b][n] x[t][f][n]      (complex, no conjugate)
//
// Per channel this is one real int8 contraction on the matrix cores,
//
//     Y (T x 2B) = U (T x 2N) . Wop (2N x 2B) - 8 . 1 colsum(Wop),
//
// where U holds the offset-binary codes u = v + 8 (0..15) of the real and
// imaginary parts of every input, column 2b + 0 of Wop holds (w_re, -w_im) and
// column 2b + 1 holds (w_im, w_re) against (u_re, u_im), and the last term,
// 8 sum_k Wop[k][c], removes the offsets exactly.
//
// The path is bound by HBM: every sample byte is read once (N bytes per time
// and channel) while the output is 8B bytes.  A workgroup takes one channel
// and 4 x TT x 32 consecutive times; consecutive workgroups take consecutive
// channels of the same times, so that together they read whole time rows of
// the frame.  Each wave streams its TT tiles of 32 times straight from global
// memory, 128 inputs (128 bytes of every row) per step with the next step's
// loads in flight (buffer loads: out-of-range reads return 0, which the zero
// weights of absent inputs and the unwritten rows of absent times make
// harmless).  The weight operands, prepared once per plan in the MFMA lane
// order, are staged per step into LDS by the whole workgroup (double
// buffered, one barrier per step), so that the four waves read them once from
// L2 between them.  A lane's A operand for one MFMA is 8 inputs of one time:
// 8 real codes, then 8 imaginary codes; in step s, k-step q (0..7), lane half
// h holds inputs 128 s + 32 (q >> 1) + 16 h + 8 (q & 1) + 0..7.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xcorr_tile.hpp"
#include "xeng_internal.hpp"

namespace xeng {
namespace {

constexpr unsigned kLow4 = 0x0F0F0F0Fu;

// Operand of k-step q (0..7) from the lane's 64 sample bytes of one step.
__device__ __forceinline__ v4i a_operand(const v4i (&raw)[4], int q) {
  const uint32_t w0 = (uint32_t)raw[q >> 1][2 * (q & 1)];
  const uint32_t w1 = (uint32_t)raw[q >> 1][2 * (q & 1) + 1];
  return v4i{(int)((w0 >> 4) & kLow4), (int)((w1 >> 4) & kLow4), (int)(w0 & kLow4),
             (int)(w1 & kLow4)};
}

// The lane's 64 sample bytes of one time and step: bytes 32 i + 16 h .. + 15
// of the step, i = 0..3 (off includes 16 h).  Aligned rows take four 16-byte
// buffer loads, others byte loads.
template <bool ALIGNED>
__device__ __forceinline__ void load_step(v4i (&raw)[4], __amdgpu_buffer_rsrc_t rs, int off) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (ALIGNED) {
      raw[i] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 32 * i, 0, 0));
    } else {
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          w |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, off + 32 * i + 4 * d + e, 0, 0)
               << (8 * e);
        raw[i][d] = (int)w;
      }
    }
  }
}

// NB: beam-component tiles (32 columns of Y each, 1..4) of this launch; TT:
// time tiles of 32 per wave.
template <int NB, int TT, bool ALIGNED>
__global__ void __launch_bounds__(256) beam_kernel(BeamArgs a) {
  __shared__ __attribute__((aligned(16))) v4i wl[2][8][NB][64];  // a step's weights, twice
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int f = logical % a.F;
  const int tb = logical / a.F;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, r = lane & 31;
  const int tbase = (tb * 4 + wave) * TT * 32;
  const long long row_stride = (long long)a.F * a.N;
  // bytes from this channel's first sample to the end of the launch's frame
  const int nrec = (int)((long long)a.T * row_stride - (long long)f * a.N);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(a.samples + (long long)f * a.N), (short)0, nrec, 0x00020000);
  const v4i* __restrict__ wop = reinterpret_cast<const v4i*>(a.wop);

  int off[TT];
#pragma unroll
  for (int j = 0; j < TT; ++j)
    off[j] = (int)((long long)(tbase + 32 * j + r) * row_stride) + 16 * h;
  // A step's weights are 8 x NB x 64 operands; thread tid stages operands
  // e = tid + 256 k, k < 2 NB, with e = (q NB + c) 64 + lane.
  auto wsrc = [&](int s, int e) {
    const int l = e & 63, c = (e >> 6) % NB, q = (e >> 6) / NB;
    return wop[((((long long)f * a.S + s) * 8 + q) * a.NBT + a.c0 + c) * 64 + l];
  };
  v4i* const wflat0 = &wl[0][0][0][0];
  v4i* const wflat1 = &wl[1][0][0][0];

  v16i acc[TT][NB];
#pragma unroll
  for (int j = 0; j < TT; ++j)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[j][c] = v16i{};

  v4i cur[TT][4], wst[2 * NB];
#pragma unroll
  for (int j = 0; j < TT; ++j) load_step<ALIGNED>(cur[j], rs, off[j]);
#pragma unroll
  for (int k = 0; k < 2 * NB; ++k) wflat0[tid + 256 * k] = wsrc(0, tid + 256 * k);
  __syncthreads();
  for (int s = 0; s < a.S; ++s) {
    v4i nxt[TT][4];
    const bool more = s + 1 < a.S;  // uniform
    const int b = s & 1;
    if (more) {
#pragma unroll
      for (int j = 0; j < TT; ++j) load_step<ALIGNED>(nxt[j], rs, off[j] + 128 * (s + 1));
#pragma unroll
      for (int k = 0; k < 2 * NB; ++k) wst[k] = wsrc(s + 1, tid + 256 * k);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      v4i W[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) W[c] = wl[b][q][c][lane];
#pragma unroll
      for (int j = 0; j < TT; ++j) {
        const v4i A = a_operand(cur[j], q);
#pragma unroll
        for (int c = 0; c < NB; ++c)
          acc[j][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, W[c], acc[j][c], 0, 0, 0);
      }
    }
    if (more) {
      // the other buffer was last read in step s - 1, before the last barrier
      v4i* const wnext = b ? wflat0 : wflat1;
#pragma unroll
      for (int k = 0; k < 2 * NB; ++k) wnext[tid + 256 * k] = wst[k];
#pragma unroll
      for (int j = 0; j < TT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) cur[j][i] = nxt[j][i];
    }
    __syncthreads();
  }

  // Y: lane holds column r of each tile and rows 8 (v >> 2) + 4 h + (v & 3)
  const int ncomp = 2 * a.B;
  const long long out_row = (long long)a.F * ncomp;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = 32 * (a.c0 + c) + r;
    if (col >= ncomp) continue;
    const int corr = a.corr[(long long)f * a.NBT * 32 + col];
    int32_t* out = a.beams + (long long)f * ncomp + col;
#pragma unroll
    for (int j = 0; j < TT; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int t = tbase + 32 * j + 8 * (v >> 2) + 4 * h + (v & 3);
        if (t < a.T) out[(long long)t * out_row] = acc[j][c][v] - corr;
      }
  }
}

template <int NB, int TT, bool ALIGNED>
hipError_t launch_nb(const BeamArgs& a, hipStream_t stream) {
  const long long grid = (long long)a.F * a.tblocks;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((beam_kernel<NB, TT, ALIGNED>), dim3((unsigned)grid), dim3(256), 0, stream,
                     a);
  return hipGetLastError();
}

// Time tiles per wave: registers hold TT x NB accumulators and two steps of
// sample operands.
constexpr int tt_of(int nb, bool aligned) { return aligned && nb <= 2 ? 2 : 1; }

template <int NB>
hipError_t launch_aligned_or_not(const BeamArgs& a, bool aligned, hipStream_t stream) {
  return aligned ? launch_nb<NB, tt_of(NB, true), true>(a, stream)
                 : launch_nb<NB, tt_of(NB, false), false>(a, stream);
}

}  // namespace

int beam_rows_per_block(int nb, bool aligned) { return 4 * 32 * tt_of(nb, aligned); }

hipError_t launch_beams(BeamArgs a, int nb, bool aligned, hipStream_t stream) {
  // a launch reads the weight operands and offset terms of component tiles
  // c0 .. c0 + nb - 1, which must lie inside the NBT tiles the plan holds
  if (nb < 1 || nb > 4 || a.c0 < 0 || a.c0 + nb > a.NBT) return hipErrorInvalidValue;
  const int rows = beam_rows_per_block(nb, aligned);
  a.tblocks = (a.T + rows - 1) / rows;
  switch (nb) {
    case 1: return launch_aligned_or_not<1>(a, aligned, stream);
    case 2: return launch_aligned_or_not<2>(a, aligned, stream);
    case 3: return launch_aligned_or_not<3>(a, aligned, stream);
    case 4: return launch_aligned_or_not<4>(a, aligned, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xeng
