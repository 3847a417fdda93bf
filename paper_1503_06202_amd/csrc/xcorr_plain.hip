// The plain correlation kernel: one workgroup per (channel, 128 x 128 tile,
// time slice) of one frame, triangular tile schedule (Sec. IV-C, "Full
// Correlation"), and the fills that clear vis before time slices add into it.
#include "xcorr_device.hpp"

namespace xeng {

template <int FORM, bool ALIGNED, bool SHIFT, bool SPLITDIAG = true>
__global__ void __launch_bounds__(NTHREADS, 2) xcorr_tile_kernel(TileArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
  // Head items first (the dispatcher issues workgroups in order), then the
  // tail items, which fill the GPU as head tiles finish.  Each phase is
  // remapped over the XCDs on its own (the head count is a multiple of 8).
  const int nhead = a.head_tiles * a.nslices;
  const int b = blockIdx.x;
  int f, p, t_begin, t_end, mode;
  if (b < nhead) {
    const int logical = xcd_logical_id(b, nhead);
    p = logical % a.tiles_per_chan;
    const int rest = logical / a.tiles_per_chan;
    const int s = rest % a.nslices;
    f = rest / a.nslices;
    t_begin = a.t0 + s * a.slice_len;
    t_end = min(a.t1, t_begin + a.slice_len);
    mode = a.write_mode;
  } else {
    const int rem = a.F * a.tiles_per_chan - a.head_tiles;
    const int k = xcd_logical_id(b - nhead, rem * a.tail_slices);
    const int g = a.head_tiles + k % rem, s = k / rem;
    f = g / a.tiles_per_chan;
    p = g % a.tiles_per_chan;
    t_begin = a.t0 + s * a.tail_len;
    t_end = min(a.t1, t_begin + a.tail_len);
    mode = a.tail_mode;
  }
  int I, J;
  tile_of(p, a.nt, I, J);
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  // int8 prefetches two chunks ahead; FP8 (wider operands, more registers)
  // and shifted frames one
  tile_body<FORM, ALIGNED, !SHIFT && FORM == FORM_I8, SHIFT, OneRange, SPLITDIAG>(
      a.samples, a.vis, a.N, a.row_stride, NB, f, I, J, OneRange{t_begin, t_end}, mode, lds,
      a.seg_delay, a.blk_delay);
}

// Fill int32 words with zero (kept out of hipMemsetAsync so that launches can
// be captured in HIP graphs).
__global__ void zero_kernel(int32_t* __restrict__ p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0;
}

// One workgroup per tile: clear the packed-triangle entries of its rows
// (row i of block I holds columns max(i, 128 J) .. min(N, 128 J + 128) - 1).
__global__ void zero_tiles_kernel(int32_t* vis, int N, int tiles_per_chan, int nt, int first) {
  const int g = first + (int)blockIdx.x;
  const int f = g / tiles_per_chan;
  int I, J;
  tile_of(g % tiles_per_chan, nt, I, J);
  const long long NB = (long long)N * (N + 1) / 2;
  int32_t* base = vis + 2 * (long long)f * NB;
  for (int r = 0; r < BT; ++r) {
    const int i = I * BT + r;
    if (i >= N) break;
    const int j0 = max(i, J * BT), j1 = min(N, J * BT + BT);
    const long long b0 = (long long)i * N - (long long)i * (i - 1) / 2 + (j0 - i);
    for (int e = threadIdx.x; e < 2 * (j1 - j0); e += blockDim.x) base[2 * b0 + e] = 0;
  }
}

hipError_t launch_zero_tiles(int32_t* vis, int N, int tiles_per_chan, int nt, int first, int count,
                             hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_tiles_kernel, dim3((unsigned)count), dim3(256), 0, stream, vis, N,
                     tiles_per_chan, nt, first);
  return hipGetLastError();
}

hipError_t launch_zero(int32_t* p, long long n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_tiles(const TileArgs& a, int form, bool aligned, hipStream_t stream) {
  const long long grid = (long long)a.head_tiles * a.nslices +
                         ((long long)a.F * a.tiles_per_chan - a.head_tiles) * a.tail_slices;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid), b(NTHREADS);
  if (!a.split_diag && aligned && !a.seg_delay) {
    // diagonal tiles keep the off-diagonal wave roles (see tile_body)
    if (form == FORM_I8)
      hipLaunchKernelGGL((xcorr_tile_kernel<FORM_I8, true, false, false>), g, b, 0, stream, a);
    else
      hipLaunchKernelGGL((xcorr_tile_kernel<FORM_F8, true, false, false>), g, b, 0, stream, a);
    return hipGetLastError();
  }
  XENG_DISPATCH3(xcorr_tile_kernel, form, aligned, a.seg_delay != nullptr, g, b, stream, a);
  return hipGetLastError();
}

}  // namespace xeng
