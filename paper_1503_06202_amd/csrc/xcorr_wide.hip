#include "xcorr_device.hpp"

namespace xeng {

// ---------------------------------------------------------------------------
// Wide tiles: 128 x 256 baselines per workgroup, one workgroup per CU.
//
// Four waves, each owning 64 x 128 baselines (2 x 4 MFMA blocks; the int32 or
// f32 accumulators fill half of the 512-register file a lone wave per SIMD
// gets).  Per MFMA this halves the barrier count and cuts LDS reads, operand
// staging and global loads by about a quarter against 128 x 128 tiles, and
// the rotated operand is built on the A side, which has two fragments per
// k-step instead of four.  Tiles (I, J) cover rows [128 I, 128 I + 128) and
// columns [256 J, 256 J + 256); the triangle needs J >= I / 2.
// ---------------------------------------------------------------------------

constexpr int WJ = 256;                      // J block width (inputs)
constexpr int PROWJ = WJ + 32;               // bytes per J plane row (padded)
constexpr int PLANE_J = KC * PROWJ;
constexpr int W_IR = 0, W_IM = PLANE, W_JR = 2 * PLANE, W_JM = 2 * PLANE + PLANE_J;
constexpr int WSTAGE = 2 * PLANE + 2 * PLANE_J;   // one buffer
constexpr int WLDS = 2 * WSTAGE;                  // double buffered

// Staging roles: I pieces (16 inputs x 1 time): seg = h & 7, rows rI + 32 k
// (k = 0, 1), rI over 0..31 in the order that keeps the two rows of a 16-lane
// write pass 4 apart; J pieces: seg = h & 15, rows (h >> 4) + 16 k (k = 0..3),
// sixteen lanes per 256-byte row.
struct WideRole {
  int segI, rI, segJ, rJ;
  __device__ __forceinline__ explicit WideRole(int h) {
    segI = h & 7;
    const int q = h >> 3;
    rI = 4 * (q & 1) + ((q >> 1) & 3) + 8 * (q >> 3);
    segJ = h & 15;
    rJ = h >> 4;
  }
};

struct WideRaw {
  v4i i[2], j[4];
};

__device__ __forceinline__ void wide_load_fast(WideRaw& raw, const uint8_t* __restrict__ rows,
                                               long long row_stride, uint32_t offI,
                                               uint32_t offJ) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
    raw.i[k] = *reinterpret_cast<const v4i*>(rows + (long long)(32 * k) * row_stride + offI);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    raw.j[k] = *reinterpret_cast<const v4i*>(rows + (long long)(16 * k) * row_stride + offJ);
}

__device__ __forceinline__ void wide_load_edge(WideRaw& raw, const uint8_t* __restrict__ samples,
                                               long long row_stride, int f, int N, int nI,
                                               int nJ, int tI, int tJ, int t_end) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
    raw.i[k] = load_piece_edge(samples, row_stride, f, N, nI, tI + 32 * k, t_end);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    raw.j[k] = load_piece_edge(samples, row_stride, f, N, nJ, tJ + 16 * k, t_end);
}

template <int FORM>
__device__ __forceinline__ void convert_piece(const v4i& w, v4i& re, v4i& im) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const uint32_t x = (uint32_t)w[d];
    const uint32_t ur = (x >> 4) & 0x0F0F0F0Fu, um = x & 0x0F0F0F0Fu;
    re[d] = (int)(FORM == FORM_I8 ? nib_to_i8(ur) : nib_to_f8(ur));
    im[d] = (int)(FORM == FORM_I8 ? nib_to_i8(um) : nib_to_f8(um));
  }
}

template <int FORM>
__device__ __forceinline__ void wide_stage(const WideRaw& raw, uint8_t* __restrict__ buf,
                                           const WideRole& sr) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    v4i re, im;
    convert_piece<FORM>(raw.i[k], re, im);
    const int off = (sr.rI + 32 * k) * PROW + 16 * sr.segI;
    *reinterpret_cast<v4i*>(buf + W_IR + off) = re;
    *reinterpret_cast<v4i*>(buf + W_IM + off) = im;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v4i re, im;
    convert_piece<FORM>(raw.j[k], re, im);
    const int off = (sr.rJ + 16 * k) * PROWJ + 16 * sr.segJ;
    *reinterpret_cast<v4i*>(buf + W_JR + off) = re;
    *reinterpret_cast<v4i*>(buf + W_JM + off) = im;
  }
}

// Transpose-read offset of this lane within a k-step for a plane of row
// pitch `prow` (see lane_read_offset).
template <int FORM>
__device__ __forceinline__ int lane_read_offset_p(int lane, int prow) {
  const int g = lane >> 4, j = lane & 15;
  const int row = (FORM == FORM_I8 ? 8 : 16) * (g >> 1) + (j >> 1);
  return row * prow + 16 * (g & 1) + 8 * (j & 1);
}

// One chunk of MFMAs of a wave's 64 x 128 sub-tile.  Re = A.B and Im = Z.B
// with A = [r_i, m_i], B = [r_j, m_j] and Z = [m_i, -r_i] per 8 samples.
template <int FORM>
__device__ __forceinline__ void wide_compute(const uint8_t* __restrict__ buf, int rdI, int rdJ,
                                             typename Acc<FORM>::T (&re)[2][4],
                                             typename Acc<FORM>::T (&im)[2][4]) {
  const uint8_t* pi = buf + rdI;
  const uint8_t* pj = buf + rdJ;
  if (FORM == FORM_I8) {
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      v4i A[2], Z[2], B[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const v2i r = lds_tr8(pi + W_IR + 16 * s * PROW + 32 * a);
        const v2i m = lds_tr8(pi + W_IM + 16 * s * PROW + 32 * a);
        A[a] = v4i{r.x, r.y, m.x, m.y};
        Z[a] = v4i{m.x, m.y, (int)neg_i8((uint32_t)r.x), (int)neg_i8((uint32_t)r.y)};
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const v2i r = lds_tr8(pj + W_JR + 16 * s * PROWJ + 32 * b);
        const v2i m = lds_tr8(pj + W_JM + 16 * s * PROWJ + 32 * b);
        B[b] = v4i{r.x, r.y, m.x, m.y};
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          re[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], B[b], re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Z[a], B[b], im[a][b], 0, 0, 0);
        }
    }
  } else {
    const int sg = (int)0x80808080u;
#pragma unroll
    for (int s = 0; s < KC / 32; ++s) {
      v8i A[2], Z[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const uint8_t* q = pi + 32 * s * PROW + 32 * a;
        const v2i r0 = lds_tr8(q + W_IR), m0 = lds_tr8(q + W_IM);
        const v2i r1 = lds_tr8(q + W_IR + 8 * PROW), m1 = lds_tr8(q + W_IM + 8 * PROW);
        A[a] = v8i{r0.x, r0.y, m0.x, m0.y, r1.x, r1.y, m1.x, m1.y};
        Z[a] = v8i{m0.x, m0.y, r0.x ^ sg, r0.y ^ sg, m1.x, m1.y, r1.x ^ sg, r1.y ^ sg};
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint8_t* q = pj + 32 * s * PROWJ + 32 * b;
        const v2i r0 = lds_tr8(q + W_JR), m0 = lds_tr8(q + W_JM);
        const v2i r1 = lds_tr8(q + W_JR + 8 * PROWJ), m1 = lds_tr8(q + W_JM + 8 * PROWJ);
        const v8i B = v8i{r0.x, r0.y, m0.x, m0.y, r1.x, r1.y, m1.x, m1.y};
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          re[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[a], B, re[a][b], 0, 0, 0,
                                                                     127, 0, 127);
          im[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(Z[a], B, im[a][b], 0, 0, 0,
                                                                     127, 0, 127);
        }
      }
    }
  }
}

template <class V>
__device__ __forceinline__ void wide_write(int32_t* vis, int N, long long NB, int f, int rs0,
                                           int cs0, int lane, int mask, int mode,
                                           V (&re)[2][4], V (&im)[2][4]) {
  int32_t* base = vis + 2 * (long long)f * NB;
#pragma unroll
  for (int ab = 0; ab < 8; ++ab) {
    const int ai = ab >> 2, bi = ab & 3;
    if (!(mask & (1 << ab))) continue;
    const int j = cs0 + 32 * bi + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = rs0 + 32 * ai + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
      if (i < N && j < N && j >= i) {
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

// Wide tile index p -> (I, J) with J >= I / 2: rows 2a and 2a + 1 hold nJ - a
// tiles each.
__device__ __forceinline__ void wide_tile_of(int p, int nI, int nJ, int& I, int& J) {
  int row = 0;
  while (row + 1 < nI && p >= nJ - (row >> 1)) {
    p -= nJ - (row >> 1);
    ++row;
  }
  I = row;
  J = (row >> 1) + p;
}

template <int FORM>
struct WideCtx {
  uint8_t* lds;
  const uint8_t* rows;
  long long row_stride;
  uint32_t offI, offJ;
  WideRole sr;
  int rdI, rdJ;
  typename Acc<FORM>::T re[2][4], im[2][4];
  __device__ __forceinline__ explicit WideCtx(int h) : sr(h) {}
};

template <int FORM, bool COMPUTE>
__device__ __forceinline__ void wide_step(WideCtx<FORM>& x, int cur, int nxt, const WideRaw& stg,
                                          WideRaw& ld, int ld_chunk) {
  wide_load_fast(ld, x.rows + (long long)ld_chunk * KC * x.row_stride, x.row_stride, x.offI,
                 x.offJ);
  __builtin_amdgcn_sched_barrier(0);
  if (COMPUTE) wide_compute<FORM>(x.lds + cur, x.rdI, x.rdJ, x.re, x.im);
  wide_stage<FORM>(stg, x.lds + nxt, x.sr);
  __syncthreads();
}

template <int FORM, bool COMPUTE>
__device__ __forceinline__ void wide_steady(WideCtx<FORM>& x, int nsteady, int nfast) {
  constexpr int B0 = 0, B1 = WSTAGE;
  WideRaw rawA, rawB;
  wide_load_fast(rawA, x.rows, x.row_stride, x.offI, x.offJ);
  wide_stage<FORM>(rawA, x.lds + B0, x.sr);
  wide_load_fast(rawA, x.rows + (long long)KC * x.row_stride, x.row_stride, x.offI, x.offJ);
  __syncthreads();
  for (int c = 0; c < nsteady; c += 2) {
    wide_step<FORM, COMPUTE>(x, B0, B1, rawA, rawB, min(c + 2, nfast - 1));
    wide_step<FORM, COMPUTE>(x, B1, B0, rawB, rawA, min(c + 3, nfast - 1));
  }
}

// One wide tile of channel f over samples [t_begin, t_end) (FP8: at most
// 65536 samples).  Requires N % 16 == 0 and 16-byte aligned rows.
template <int FORM>
__device__ __forceinline__ void wide_body(const uint8_t* __restrict__ samples, int32_t* vis,
                                          int N, long long row_stride, long long NB, int f,
                                          int I, int J, int t_begin, int t_end, int mode,
                                          uint8_t* lds) {
  const int len = t_end > t_begin ? t_end - t_begin : 0;
  const int nchunks = (len + KC - 1) / KC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int rs0 = I * BT + 64 * wr, cs0 = J * WJ + 128 * wc;
  int mask = 0;
#pragma unroll
  for (int ab = 0; ab < 8; ++ab) {
    const int rs = rs0 + 32 * (ab >> 2), cs = cs0 + 32 * (ab & 3);
    if (rs < N && cs < N && cs >= rs) mask |= 1 << ab;
  }
  WideCtx<FORM> x(tid);
  const int nI = I * BT + 16 * x.sr.segI, nJ = J * WJ + 16 * x.sr.segJ;
  const uint8_t* rows = samples + (long long)t_begin * row_stride + (long long)f * N;
  x.lds = lds;
  x.rows = rows;
  x.row_stride = row_stride;
  x.offI = (uint32_t)x.sr.rI * (uint32_t)row_stride + (uint32_t)(nI < N ? nI : 0);
  x.offJ = (uint32_t)x.sr.rJ * (uint32_t)row_stride + (uint32_t)(nJ < N ? nJ : 0);
  x.rdI = lane_read_offset_p<FORM>(lane, PROW) + 64 * wr;
  x.rdJ = lane_read_offset_p<FORM>(lane, PROWJ) + 128 * wc;
  typedef typename Acc<FORM>::T V;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x.re[p][q] = V{};
      x.im[p][q] = V{};
    }
  const int nfast = len / KC;
  const int nsteady = nfast & ~1;
  int c = 0;
  if (nsteady >= 2) {
    if (mask)
      wide_steady<FORM, true>(x, nsteady, nfast);
    else
      wide_steady<FORM, false>(x, nsteady, nfast);
    c = nsteady;
  }
  // remaining chunks (ragged tail, short ranges): one buffer flip per chunk
  WideRaw raw;
  auto load = [&](int cc) {
    if ((cc + 1) * KC <= len)
      wide_load_fast(raw, rows + (long long)cc * KC * row_stride, row_stride, x.offI, x.offJ);
    else
      wide_load_edge(raw, samples, row_stride, f, N, nI, nJ, t_begin + cc * KC + x.sr.rI,
                     t_begin + cc * KC + x.sr.rJ, t_end);
  };
  if (c < nchunks) {
    load(c);
    wide_stage<FORM>(raw, lds + (c & 1) * WSTAGE, x.sr);
    __syncthreads();
  }
  for (; c < nchunks; ++c) {
    uint8_t* cur = lds + (c & 1) * WSTAGE;
    uint8_t* nxt = lds + ((c + 1) & 1) * WSTAGE;
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    if (mask) wide_compute<FORM>(cur, x.rdI, x.rdJ, x.re, x.im);
    if (more) wide_stage<FORM>(raw, nxt, x.sr);
    __syncthreads();
  }
  if (mask) wide_write(vis, N, NB, f, rs0, cs0, lane, mask, mode, x.re, x.im);
}

template <int FORM>
__global__ void __launch_bounds__(NTHREADS, 1) xcorr_wide_kernel(TileArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[WLDS];
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int p = logical % a.tiles_per_chan;
  const int rest = logical / a.tiles_per_chan;
  const int s = rest % a.nslices;
  const int f = rest / a.nslices;
  int I, J;
  wide_tile_of(p, a.nt, (a.N + WJ - 1) / WJ, I, J);
  const int t_begin = a.t0 + s * a.slice_len;
  const int t_end = min(a.t1, t_begin + a.slice_len);
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  wide_body<FORM>(a.samples, a.vis, a.N, a.row_stride, NB, f, I, J, t_begin, t_end,
                  a.write_mode, lds);
}

hipError_t launch_wide(const TileArgs& a, int form, hipStream_t stream) {
  const long long grid = (long long)a.F * a.tiles_per_chan * a.nslices;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid), b(NTHREADS);
  if (form == FORM_I8)
    hipLaunchKernelGGL((xcorr_wide_kernel<FORM_I8>), g, b, 0, stream, a);
  else
    hipLaunchKernelGGL((xcorr_wide_kernel<FORM_F8>), g, b, 0, stream, a);
  return hipGetLastError();
}

}  // namespace xeng
