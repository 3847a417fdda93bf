// Time shifting by a shifted copy of the frame (Sec. IV-C, "Time Shifting").
//
// The correlation kernels apply a delay per 16-input group in their loads,
// which costs nothing while the eight groups of a 128-input block share their
// delay (a row piece of the block is still one 128-byte line).  Delays that
// differ inside a block make every group of a line a line of its own, and the
// tiles that read a block no longer share lines in L2.  For such delays the
// frame is first copied, shifted, into a plan-owned buffer:
//
//     dst[t][f][16 g + e] = src[t - d_g][f][16 g + e],   0 <= t < T,
//
// where rows t - d_g < 0 are the history before src; the correlation then
// reads the copy with no delay.  One thread per 16-input piece.  Every
// 16-byte read fetches a whole 128-byte line, whose other seven pieces the
// copy needs again at other output rows, up to the largest delay later.  The
// copy therefore runs over one line column (eight groups of one channel) at a
// time, all output rows of the column together: eight neighbouring threads
// write one output line, and a line read for one group of the column is
// more often still cached (in the memory-side cache) when the column's other
// groups read it than when every channel's rows are copied in turn.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xeng_internal.hpp"

namespace xeng {
namespace {

template <bool VEC>
__global__ void __launch_bounds__(256) shift_copy_kernel(const uint8_t* __restrict__ src,
                                                         uint8_t* __restrict__ dst, int N, int F,
                                                         int T, const int* __restrict__ seg_delay) {
  const int P = (N + 15) / 16;
  const int C = (P + 7) / 8;  // line columns of a channel
  // e = ((f C + c) T + t) 8 + g: piece p = 8 c + g of row t of channel f
  const long long total = (long long)F * C * T * 8;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int g = (int)(e & 7);
    const long long rest = e >> 3;
    const long long t = rest % T, fc = rest / T;
    const int c = (int)(fc % C), f = (int)(fc / C);
    const int p = 8 * c + g;
    if (p >= P) continue;  // the last column of a channel whose N is not a multiple of 128
    const long long from = ((t - seg_delay[p]) * F + f) * N + 16 * p;
    const long long to = (t * F + f) * N + 16 * p;
    if (VEC) {
      *reinterpret_cast<uint4*>(dst + to) = *reinterpret_cast<const uint4*>(src + from);
    } else {
      const int n = N - 16 * p < 16 ? N - 16 * p : 16;
      for (int b = 0; b < n; ++b) dst[to + b] = src[from + b];
    }
  }
}

}  // namespace

hipError_t launch_shift_copy(const uint8_t* src, uint8_t* dst, int N, int F, int T,
                             const int* seg_delay, hipStream_t stream) {
  const long long total = (long long)F * ((N + 127) / 128) * T * 8;
  if (total <= 0) return hipSuccess;
  long long blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  const bool vec = (N % 16 == 0) && ((reinterpret_cast<uintptr_t>(src) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(dst) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL(shift_copy_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, src,
                       dst, N, F, T, seg_delay);
  else
    hipLaunchKernelGGL(shift_copy_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, src,
                       dst, N, F, T, seg_delay);
  return hipGetLastError();
}

}  // namespace xeng
