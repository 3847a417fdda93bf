// The batched persistent correlation kernel: many instances in one launch.
#include "xcorr_device.hpp"

namespace xeng {

// Persistent batched kernel: every workgroup takes work items from a global
// counter until the list is exhausted (every workgroup reaches the exit).
// Items are sorted by decreasing cost on the host, so the tail is short.
template <int FORM>
__global__ void __launch_bounds__(NTHREADS, 2)
    xcorr_batch_kernel(const BatchInst* __restrict__ insts, const BatchItem* __restrict__ items,
                       int nitems, int* counter) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
  // the next work item's index travels through the first LDS word, which is
  // free between tiles (the LDS budget of two workgroups per CU is exact)
  int* next = reinterpret_cast<int*>(lds);
  for (;;) {
    if (threadIdx.x == 0) *next = atomicAdd(counter, 1);
    __syncthreads();
    const int k = *next;
    __syncthreads();  // every thread has read it before the LDS is reused
    if (k >= nitems) break;
    const BatchItem it = items[k];
    const BatchInst in = insts[it.inst];
    if (!in.samples) continue;  // instance not active in this call (uniform branch)
    const long long NB = (long long)in.N * (in.N + 1) / 2;
    const long long stride = (long long)in.F * in.N;
    // int8 prefetches two chunks ahead on the fast path (as the plain kernel
    // does); FP8 one
    // (64-bit atomic adds for the tiles of time-sliced instances)
    if (in.aligned)
      tile_body<FORM, true, FORM == FORM_I8, false, OneRange, true, true>(
          in.samples, in.vis, in.N, stride, NB, it.f, it.I, it.J, OneRange{it.t0, it.t1}, it.mode,
          lds);
    else
      tile_body<FORM, false, false, false, OneRange, true, true>(
          in.samples, in.vis, in.N, stride, NB, it.f, it.I, it.J, OneRange{it.t0, it.t1}, it.mode,
          lds);
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

}  // namespace xeng
