// X-engine correlation kernels for gfx950: one workgroup per (channel, tile of
// 128 x 128 baselines, time slice), triangular tile schedule, int8 or FP8 MFMA.
//
// What is computed: V_f[i][j] = sum_t x_i conj(x_j) over the upper triangle
// including the diagonal (Sec. I; Sec. IV-C, "Full Correlation"; the baseline
// count N(N+1)/2 of Eq. (1)), on 4+4-bit offset-binary samples (Sec. II-A,
// footnote).  The tile layout, the operand packing and the MFMA formulation are
// described in xcorr_tile.hpp.
#include "xcorr_tile.hpp"
#include "xeng_internal.hpp"

namespace xeng {

// One 64-sample chunk of an 8 x 8 block: raw[k] holds the bytes of inputs
// n0..n0+7 at time t0 + k (x: n0..n0+3, y: n0+4..n0+7).
template <bool ALIGNED>
__device__ __forceinline__ void load_chunk(uint2 (&raw)[8], const uint8_t* __restrict__ samples,
                                           long long row_stride, int f, int N, int n0, int t0,
                                           int t_end, bool active) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int t = t0 + k;
    raw[k] = make_uint2(0x88888888u, 0x88888888u);  // the code of 0 + 0i
    if (active && t < t_end && n0 < N) {
      const uint8_t* p = samples + (long long)t * row_stride + (long long)f * N + n0;
      if (ALIGNED) {
        raw[k] = *reinterpret_cast<const uint2*>(p);
      } else {
        uint32_t w[2] = {0x88888888u, 0x88888888u};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (n0 + e < N) {
            const uint32_t sh = 8 * (e & 3);
            w[e >> 2] = (w[e >> 2] & ~(0xFFu << sh)) | ((uint32_t)p[e] << sh);
          }
        }
        raw[k] = make_uint2(w[0], w[1]);
      }
    }
  }
}

// Transpose the 8 x 8 byte block, split nibbles, convert and store the 8 rows'
// segment q into an LDS operand block.
template <int FORM>
__device__ __forceinline__ void stage_chunk(uint2 (&raw)[8], uint8_t* __restrict__ blk,
                                            int row0, int q) {
  transpose4x4(raw[0].x, raw[1].x, raw[2].x, raw[3].x);
  transpose4x4(raw[4].x, raw[5].x, raw[6].x, raw[7].x);
  transpose4x4(raw[0].y, raw[1].y, raw[2].y, raw[3].y);
  transpose4x4(raw[4].y, raw[5].y, raw[6].y, raw[7].y);
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const uint32_t lo = n < 4 ? raw[n].x : raw[n - 4].y;  // times 0..3
    const uint32_t hi = n < 4 ? raw[n + 4].x : raw[n].y;  // times 4..7
    const uint32_t rl = (lo >> 4) & 0x0F0F0F0Fu, rh = (hi >> 4) & 0x0F0F0F0Fu;
    const uint32_t ml = lo & 0x0F0F0F0Fu, mh = hi & 0x0F0F0F0Fu;
    v4i seg;
    if (FORM == FORM_I8) {
      seg = v4i{(int)nib_to_i8(rl), (int)nib_to_i8(rh), (int)nib_to_i8(ml), (int)nib_to_i8(mh)};
    } else {
      seg = v4i{(int)nib_to_f8(rl), (int)nib_to_f8(rh), (int)nib_to_f8(ml), (int)nib_to_f8(mh)};
    }
    *reinterpret_cast<v4i*>(blk + seg_off(row0 + n, q)) = seg;
  }
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

// One chunk of MFMAs for a wave's 64 x 64 sub-tile (2 x 2 blocks of 32 x 32).
// mask bit (2a + b) enables block (a, b).
template <int FORM>
__device__ __forceinline__ void compute_chunk(const uint8_t* __restrict__ ldsI,
                                              const uint8_t* __restrict__ ldsJ, int ra, int rb,
                                              int half, int mask,
                                              typename Acc<FORM>::T (&re)[2][2],
                                              typename Acc<FORM>::T (&im)[2][2]) {
  if (FORM == FORM_I8) {
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      const int q = 2 * s + half;
      v4i A[2], B[2], Y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) A[a] = *reinterpret_cast<const v4i*>(ldsI + seg_off(ra + 32 * a, q));
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        B[b] = *reinterpret_cast<const v4i*>(ldsJ + seg_off(rb + 32 * b, q));
        // [r r m m] -> [-m -m r r]
        Y[b] = v4i{(int)neg_i8((uint32_t)B[b].z), (int)neg_i8((uint32_t)B[b].w), B[b].x, B[b].y};
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (mask & (1 << (2 * a + b))) {
            re[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], B[b], re[a][b], 0, 0, 0);
            im[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], Y[b], im[a][b], 0, 0, 0);
          }
    }
  } else {
#pragma unroll
    for (int s = 0; s < KC / 32; ++s) {
      const int q0 = 4 * s + 2 * half;
      v8i A[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const v4i x0 = *reinterpret_cast<const v4i*>(ldsI + seg_off(ra + 32 * a, q0));
        const v4i x1 = *reinterpret_cast<const v4i*>(ldsI + seg_off(ra + 32 * a, q0 + 1));
        A[a] = v8i{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const v4i x0 = *reinterpret_cast<const v4i*>(ldsJ + seg_off(rb + 32 * b, q0));
        const v4i x1 = *reinterpret_cast<const v4i*>(ldsJ + seg_off(rb + 32 * b, q0 + 1));
        const v8i B = v8i{x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        // FP8 negation flips the sign bit: [r r m m] -> [-m -m r r]
        const int sg = (int)0x80808080u;
        const v8i Y = v8i{x0.z ^ sg, x0.w ^ sg, x0.x, x0.y, x1.z ^ sg, x1.w ^ sg, x1.x, x1.y};
#pragma unroll
        for (int a = 0; a < 2; ++a)
          if (mask & (1 << (2 * a + b))) {
            // format 0 = FP8 e4m3 for both operands; scale exponent 127 = 2^0
            re[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[a], B, re[a][b], 0, 0, 0,
                                                                       127, 0, 127);
            im[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[a], Y, im[a][b], 0, 0, 0,
                                                                       127, 0, 127);
          }
      }
    }
  }
}

__device__ __forceinline__ int to_i32(int x) { return x; }
__device__ __forceinline__ int to_i32(float x) { return (int)x; }  // exact: integral, |x| < 2^24

// Write a wave's finished blocks into the packed triangle.  Offsets within a
// channel are 32-bit (the plan limits N so that 2 N(N+1)/2 < 2^31).
template <class V>
__device__ __forceinline__ void write_blocks(int32_t* vis, int N, long long NB, int f, int rs0,
                                             int cs0, int lane, int mask, int mode,
                                             V (&re)[2][2], V (&im)[2][2]) {
  int32_t* base = vis + 2 * (long long)f * NB;
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int ai = ab >> 1, bi = ab & 1;
    if (!(mask & (1 << ab))) continue;
    const int j = cs0 + 32 * bi + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = rs0 + 32 * ai + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      if (i < N && j < N && j >= i) {
        // b(i, j) = i N - i (i - 1) / 2 + (j - i)
        const int b = i * N - ((i * (i - 1)) >> 1) + (j - i);
        int32_t* p = base + 2 * b;
        const int vr = to_i32(re[ai][bi][v]);
        const int vi = (i == j) ? 0 : to_i32(im[ai][bi][v]);
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

// Map a linear workgroup id to (channel, slice, tile) so that consecutive
// logical ids, which share input rows, run on the same XCD: the dispatcher
// deals workgroups to the 8 XCDs round robin.
__device__ __forceinline__ int xcd_logical_id(int b, int G) {
  const int xcd = b & 7, slot = b >> 3, q = G >> 3, r = G & 7;
  return xcd * q + (xcd < r ? xcd : r) + slot;
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

// The work of one tile: baselines [I*128, I*128+128) x [J*128, J*128+128) of
// channel f, integrated over samples [t_begin, t_end).  All 256 threads call
// it; it ends with the tile written (mode) and the LDS free for reuse.
// FP8 form: the caller keeps t_end - t_begin <= 65536, so that every f32
// partial sum is an integer of magnitude <= 128 * 65536 = 2^23 (exact).
template <int FORM, bool ALIGNED>
__device__ __forceinline__ void tile_body(const uint8_t* __restrict__ samples, int32_t* vis,
                                          int N, long long row_stride, long long NB, int f,
                                          int I, int J, int t_begin, int t_end, int mode,
                                          uint8_t* lds) {
  const bool diag = (I == J);
  const int nchunks = t_end > t_begin ? (t_end - t_begin + KC - 1) / KC : 0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, half = lane >> 5;

  // MFMA blocks of this wave that hold baselines of the triangle
  const int rs0 = I * BT + 64 * wr, cs0 = J * BT + 64 * wc;
  int mask = 0;
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int rs = rs0 + 32 * (ab >> 1), cs = cs0 + 32 * (ab & 1);
    if (rs < N && cs < N && cs >= rs) mask |= 1 << ab;
  }

  // staging role: threads 0..127 load the I block, 128..255 the J block
  const int sblk = tid >> 7, h = tid & 127, ng = h & 15, tg = h >> 4;
  const bool sactive = (sblk == 0) || !diag;
  const int n0 = (sblk ? J : I) * BT + 8 * ng;

  typedef typename Acc<FORM>::T V;
  V re[2][2], im[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      re[x][y] = V{};
      im[x][y] = V{};
    }

  uint2 raw[8];
  if (nchunks > 0) {
    load_chunk<ALIGNED>(raw, samples, row_stride, f, N, n0, t_begin + 8 * tg, t_end, sactive);
    if (sactive) stage_chunk<FORM>(raw, lds + sblk * BLOCK_LDS, 8 * ng, tg);
  }
  __syncthreads();

  for (int c = 0; c < nchunks; ++c) {
    uint8_t* cur = lds + (c & 1) * STAGE_LDS;
    uint8_t* nxt = lds + ((c + 1) & 1) * STAGE_LDS;
    const bool more = c + 1 < nchunks;
    if (more)
      load_chunk<ALIGNED>(raw, samples, row_stride, f, N, n0, t_begin + (c + 1) * KC + 8 * tg,
                          t_end, sactive);
    if (mask) {
      const uint8_t* ldsI = cur;
      const uint8_t* ldsJ = diag ? cur : cur + BLOCK_LDS;
      compute_chunk<FORM>(ldsI, ldsJ, 64 * wr + (lane & 31), 64 * wc + (lane & 31), half, mask,
                          re, im);
    }
    if (more && sactive) stage_chunk<FORM>(raw, nxt + sblk * BLOCK_LDS, 8 * ng, tg);
    __syncthreads();
  }
  if (mask) write_blocks(vis, N, NB, f, rs0, cs0, lane, mask, mode, re, im);
}

template <int FORM, bool ALIGNED>
__global__ void __launch_bounds__(NTHREADS, 2) xcorr_tile_kernel(TileArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int p = logical % a.tiles_per_chan;
  const int rest = logical / a.tiles_per_chan;
  const int s = rest % a.nslices;
  const int f = rest / a.nslices;
  int I, J;
  tile_of(p, a.nt, I, J);
  const int t_begin = a.t0 + s * a.slice_len;
  const int t_end = min(a.t1, t_begin + a.slice_len);
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  tile_body<FORM, ALIGNED>(a.samples, a.vis, a.N, a.row_stride, NB, f, I, J, t_begin, t_end,
                           a.write_mode, lds);
}

// Persistent batched kernel: every workgroup takes work items from a global
// counter until the list is exhausted (every workgroup reaches the exit).
// Items are sorted by decreasing cost on the host, so the tail is short.
template <int FORM>
__global__ void __launch_bounds__(NTHREADS, 2)
    xcorr_batch_kernel(const BatchInst* __restrict__ insts, const BatchItem* __restrict__ items,
                       int nitems, int* counter) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int k = next;
    __syncthreads();  // every thread has read `next` before thread 0 rewrites it
    if (k >= nitems) break;
    const BatchItem it = items[k];
    const BatchInst in = insts[it.inst];
    const long long NB = (long long)in.N * (in.N + 1) / 2;
    const long long stride = (long long)in.F * in.N;
    if (in.aligned)
      tile_body<FORM, true>(in.samples, in.vis, in.N, stride, NB, it.f, it.I, it.J, it.t0, it.t1,
                            it.mode, lds);
    else
      tile_body<FORM, false>(in.samples, in.vis, in.N, stride, NB, it.f, it.I, it.J, it.t0, it.t1,
                             it.mode, lds);
  }
}

// Before a batch launch: reset the work counter and zero the outputs of the
// instances whose tiles are integrated by several slices (atomic adds).
__global__ void batch_prep_kernel(const BatchInst* __restrict__ insts, int ninst, int* counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  for (int k = 0; k < ninst; ++k) {
    const BatchInst in = insts[k];
    if (!in.zero) continue;
    const long long n = (long long)in.F * in.N * (in.N + 1);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
      in.vis[i] = 0;
  }
}

// Fill int32 words with zero (kept out of hipMemsetAsync so that launches can
// be captured in HIP graphs).
__global__ void zero_kernel(int32_t* __restrict__ p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}

hipError_t launch_zero(int32_t* p, long long n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchInst* insts, int ninst, const BatchItem* items, int nitems,
                        int* counter, int grid, int form, bool any_zero, hipStream_t stream) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_prep_kernel, dim3(any_zero ? 2048 : 1), dim3(256), 0, stream, insts,
                     ninst, counter);
  if (form == FORM_I8)
    hipLaunchKernelGGL((xcorr_batch_kernel<FORM_I8>), dim3(grid), dim3(NTHREADS), 0, stream,
                       insts, items, nitems, counter);
  else
    hipLaunchKernelGGL((xcorr_batch_kernel<FORM_F8>), dim3(grid), dim3(NTHREADS), 0, stream,
                       insts, items, nitems, counter);
  return hipGetLastError();
}

hipError_t launch_tiles(const TileArgs& a, int form, bool aligned, hipStream_t stream) {
  const long long grid = (long long)a.F * a.tiles_per_chan * a.nslices;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid), b(NTHREADS);
  if (form == FORM_I8) {
    if (aligned)
      hipLaunchKernelGGL((xcorr_tile_kernel<FORM_I8, true>), g, b, 0, stream, a);
    else
      hipLaunchKernelGGL((xcorr_tile_kernel<FORM_I8, false>), g, b, 0, stream, a);
  } else {
    if (aligned)
      hipLaunchKernelGGL((xcorr_tile_kernel<FORM_F8, true>), g, b, 0, stream, a);
    else
      hipLaunchKernelGGL((xcorr_tile_kernel<FORM_F8, false>), g, b, 0, stream, a);
  }
  return hipGetLastError();
}

}  // namespace xeng

