// The gated correlation kernel (Sec. IV-C, "Output Gating").
#include "xcorr_device.hpp"

namespace xeng {

// Output gating (Sec. IV-C, "Output Gating"): the output is partitioned into
// G sub-buffers by the time of each sample.  One workgroup per (channel,
// tile, work gate) integrates all runs of its work gate, carrying its
// accumulators and sums across runs, and writes its tile once: the samples
// are read once in all.  A work gate is a whole gate, written without
// atomics, unless that gate's runs hold more chunk-rounded samples than one
// exact integration may: the host then splits it into work gates that add
// atomically (GatedArgs).  Consecutive logical ids are the tiles of one
// (work gate, channel), which share samples.
template <int FORM, bool ALIGNED, bool SHIFT>
__global__ void __launch_bounds__(NTHREADS, 2) xcorr_gated_kernel(GatedArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int p = logical % a.tiles_per_chan;
  const int rest = logical / a.tiles_per_chan;
  const int f = rest % a.F;
  const int g = rest / a.F;
  int I, J;
  tile_of(p, a.nt, I, J);
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  const int r0 = a.gate_off[g], r1 = a.gate_off[g + 1];
  if (a.skip_empty && r1 == r0) return;  // uniform over the workgroup, before any barrier
  // a work item may stand for part of a gate's runs: it then writes into that
  // gate's buffer, in its own write mode (see GatedArgs)
  const int2 vg = a.vgate ? a.vgate[g] : make_int2(g, a.write_mode);
  tile_body<FORM, ALIGNED, false, SHIFT>(a.samples, a.vis + (long long)vg.x * a.F * NB * 2, a.N,
                                         a.row_stride, NB, f, I, J,
                                         RunList{a.runs + r0, r1 - r0}, vg.y, lds, a.seg_delay,
                                         a.blk_delay);
}

hipError_t launch_gated(const GatedArgs& a, int form, bool aligned, hipStream_t stream) {
  const long long grid = (long long)a.F * a.tiles_per_chan * a.G;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid), b(NTHREADS);
  XENG_DISPATCH3(xcorr_gated_kernel, form, aligned, a.seg_delay != nullptr, g, b, stream, a);
  return hipGetLastError();
}

}  // namespace xeng
