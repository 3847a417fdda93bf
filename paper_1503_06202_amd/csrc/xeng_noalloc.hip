// Batched correlation for callers that cannot allocate: the instance table,
// the work list and the work counter of the persistent batch kernel live in a
// file-scope device array instead of plan-owned memory.
#include "xcorr_device.hpp"
#include "xeng_noalloc.hpp"

#include <mutex>

namespace xeng {

// The library's fixed workspace: one copy per GPU, held until the process
// ends.  Every call on a GPU shares it, so calls that overlap on one GPU race.
// Host code must not pass `scratch` itself to a kernel (on the host it is a
// stand-in, not a device address): it uses the address that scratch_address
// returns.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_addr[kMaxDevices] = {};
int g_cus[kMaxDevices] = {};

// Build the instance table and the work list in the workspace from the
// descriptors passed by value.  Work item i belongs to the instance k with
// inst[k].first <= i < inst[k + 1].first; within it, l = i - first runs over
// (channel, tile, slice) with the slices of a tile adjacent.
__global__ void noalloc_prep_kernel(NoallocArgs a) {
  BatchInst* insts = reinterpret_cast<BatchInst*>(a.ws + kNoallocInstOff);
  BatchItem* items = reinterpret_cast<BatchItem*>(a.ws + kNoallocItemsOff);
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < a.ninst) {
    const NoallocInst& in = a.inst[gid];
    BatchInst b;
    b.samples = in.samples;
    b.vis = in.vis;
    b.N = in.N;
    b.F = in.F;
    b.T = in.T;
    b.aligned = (in.flags >> 3) & 1;
    b.zero = (in.flags >> 2) & 1;
    b.pad = 0;
    insts[gid] = b;
  }
  for (int i = gid; i < a.nitems; i += gridDim.x * blockDim.x) {
    int k = 0;
    while (k + 1 < a.ninst && a.inst[k + 1].first <= i) ++k;
    const NoallocInst& in = a.inst[k];
    const int l = i - in.first;
    const int s = l % in.S, rest = l / in.S;
    const int nt = (in.N + BT - 1) / BT, tpc = nt * (nt + 1) / 2;
    BatchItem it;
    it.inst = k;
    it.f = rest / tpc;
    tile_of(rest % tpc, nt, it.I, it.J);
    it.t0 = s * in.len;
    it.t1 = min(in.T, (s + 1) * in.len);
    it.mode = in.flags & 3;
    it.pad = 0;
    items[i] = it;
  }
}

}  // namespace

hipError_t noalloc_workspace(unsigned char** addr, int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  if (dev >= 0 && dev < kMaxDevices && g_addr[dev]) {
    *addr = g_addr[dev];
    *cus = g_cus[dev];
    return hipSuccess;
  }
  // once per device, with that device current: each GPU holds its own copy
  // of the array at its own address
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  int n = 0;
  e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *addr = static_cast<unsigned char*>(p);
  *cus = n > 0 ? n : 1;
  if (dev >= 0 && dev < kMaxDevices) {
    g_addr[dev] = *addr;
    g_cus[dev] = *cus;
  }
  return hipSuccess;
}

hipError_t launch_noalloc_prep(const NoallocArgs& a, hipStream_t stream) {
  const int threads = 256;
  int blocks = (a.nitems + threads - 1) / threads;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(noalloc_prep_kernel, dim3(blocks), dim3(threads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace xeng
