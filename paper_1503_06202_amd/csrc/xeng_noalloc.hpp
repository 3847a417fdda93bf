// Layout of the fixed workspace behind xeng_correlate_batch_noalloc, and the
// descriptors its preparation kernel takes by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "xeng.h"
#include "xeng_internal.hpp"

namespace xeng {

// [0, 256): the work counter; [256, 4096): the instance table (BatchInst);
// [4096, ...): the work list (BatchItem).
constexpr size_t kNoallocInstOff = 256;
constexpr size_t kNoallocItemsOff = 4096;
constexpr size_t kNoallocScratchBytes =
    kNoallocItemsOff + (size_t)XENG_NOALLOC_ITEMS_MAX * sizeof(BatchItem);
static_assert(kNoallocInstOff + XENG_NOALLOC_INST_MAX * sizeof(BatchInst) <= kNoallocItemsOff,
              "instance table overlaps the work list");

// One instance as the preparation kernel sees it (passed in the kernel's
// arguments, which stay below 4 KiB).
struct NoallocInst {
  const uint8_t* samples;  // device [T][F][N]
  int32_t* vis;            // device [F][N(N+1)/2][2]
  int N, F, T;
  int S, len;   // time slices per tile and samples per slice (a multiple of 64)
  int flags;    // bits 0-1 write mode, bit 2 clear vis first, bit 3 fast loads
  int first;    // index of its first work item
  int pad;
};

struct NoallocArgs {
  unsigned char* ws;  // the workspace's device address (from noalloc_workspace)
  int ninst, nitems;
  NoallocInst inst[XENG_NOALLOC_INST_MAX];
};
static_assert(sizeof(NoallocArgs) <= 4096, "kernel arguments above 4 KiB");

// The workspace's device address on the current device (looked up once per
// device) and that device's compute units.
hipError_t noalloc_workspace(unsigned char** addr, int* cus);
// Write the instance table and the work list into the workspace.
hipError_t launch_noalloc_prep(const NoallocArgs& a, hipStream_t stream);

}  // namespace xeng
