// Interface between the C ABI (xeng_api.cpp) and the channel kernel
// (xcorr_chan.hip).
#pragma once

#include "xeng_internal.hpp"

namespace xeng {

// Arguments of the channel kernel (int8, N <= 256): one workgroup per
// (channel f, time slice s), integrating [t0 + s slice_len, ...) within
// [t0, t1) into the whole triangle of channel f.
struct ChanArgs {
  const uint8_t* samples;  // device [T][F][N]
  int32_t* vis;            // device [F][N(N+1)/2][2]
  int N, F;
  int t0, t1;
  int nslices, slice_len;  // slice_len a multiple of 64
  int write_mode;          // WM_STORE or WM_ADD into vis; WM_STORE into partial
  long long row_stride;    // F * N
  // with several slices: slice s stores its own sums into
  // partial + s F N(N+1) (same layout as vis), for launch_chan_reduce
  int32_t* partial;
};

// aligned: fast 16-byte loads (N % 16 == 0, 16-byte aligned rows, F N <= 2^25)
hipError_t launch_chan(const ChanArgs& a, bool aligned, hipStream_t stream);

// vis[i] (+)= sum over s < ns of partial[s n + i], i < n (add: accumulate)
hipError_t launch_chan_reduce(const int32_t* partial, int32_t* vis, long long n, int ns, bool add,
                              hipStream_t stream);

}  // namespace xeng
