// C ABI of the X-engine (declared in include/xeng.h): plans, argument checks,
// launch configuration and the batched form's work lists and graphs.
//
// Every check that can fail on arguments runs on the host before the first
// HIP call, so those errors are reported the same with or without a GPU.
#include "xeng.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "xeng_chan.hpp"
#include "xeng_internal.hpp"
#include "xeng_noalloc.hpp"

namespace {

constexpr int kTile = 128;   // tile edge of the kernels
constexpr int kChunk = 64;   // samples per staged chunk
constexpr int kOccupancy = 2;  // workgroups per CU (LDS: 64 KiB each)
constexpr int kChanMax = 2 * kTile;  // inputs of the channel kernel
// Output gating: extra work gates one launch segment can need when gates are
// split (fewer than 2 x 64 = 128; see xeng_correlate_gated).
constexpr int kSplitMax = 128;
constexpr int kStageRing = 4;  // pinned staging copies of a batch plan's instance table

enum PlanKind { PLAN_SINGLE = 1, PLAN_BATCH = 2 };

}  // namespace

struct xeng_plan_s {
  int kind = 0;
  int N = 0, F = 0, T_max = 0;
  unsigned flags = 0;
  int form = XENG_FORM_I8;
  bool accumulate = false;
  int split_t = 0;  // 0 = automatic
  int kernel = 0;   // 0 = automatic, 1 = 128 x 128 tiles, 2 = 128 x 256 tiles,
                    // 3 / 4 = 128 x 128 tiles with split / common diagonal roles
  int cu_count = 0;
  std::string err;

  // batched form
  std::vector<xeng_instance> insts;
  std::vector<xeng::BatchItem> items;
  std::vector<int> inst_zero;
  bool any_zero = false;
  // pinned staging of the instance table: a ring of kStageRing copies, so
  // that a call refills one while earlier calls' uploads are still queued
  xeng::BatchInst* h_insts = nullptr;
  xeng::BatchInst* d_insts = nullptr;
  xeng::BatchItem* d_items = nullptr;
  int* d_counter = nullptr;
  hipEvent_t copy_done[kStageRing] = {};
  bool copy_pending[kStageRing] = {};
  int stage_next = 0;
  std::vector<const void*> uploaded;  // pointers now in d_insts
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t capture_stream = nullptr;

  // output gating (xeng_plan_gated): run tables, pinned staging and device
  int G_max = 0;
  long long gate_off_cap = 0, runs_cap = 0, vgate_cap = 0;  // entries
  int* h_gate_off = nullptr;
  int2* h_runs = nullptr;
  int2* h_vgate = nullptr;
  int* d_gate_off = nullptr;
  int2* d_runs = nullptr;
  int2* d_vgate = nullptr;
  hipEvent_t gate_done = nullptr;
  bool gate_pending = false;
  std::vector<int> gate_count, gate_fill;  // host work space of the run tables, G_max each
  std::vector<int> gate_zero;              // gates to clear before a split gate adds into them
  std::vector<int> seg_goff, seg_nvg;      // per launch segment: first table entry, work gates

  // channel kernel with time slices: the slices' partial triangles (plan-owned,
  // grown on demand) and the event of the last call that read them
  int32_t* d_chan_ws = nullptr;
  size_t chan_ws_ints = 0;
  hipEvent_t chan_ws_used = nullptr;
  bool chan_ws_pending = false;

  // time shifting (xeng_plan_set_delays): per-segment delays and block maxima
  bool shift = false;
  int* d_seg_delay = nullptr;
  int* d_blk_delay = nullptr;
  // delays that differ inside a 128-input block: shifted copy of the frame
  bool shift_copy = false;
  uint8_t* d_shifted = nullptr;

  // flagged data (xeng_plan_flagged): event frame, its correlation and counters
  bool flagged = false;
  long long flag_cap = 0;  // event rows per channel
  int flag_nseg = 0;       // launch segments of the event correlation
  uint8_t* d_fU = nullptr;
  int32_t* d_fX = nullptr;
  int* d_fint = nullptr;   // cnt [F], single [F N], n [F N], R [1], gate_off [2 nseg]
  int2* d_fruns = nullptr;

  // The delay tables and the beam weight operands are replaced only after the
  // plan's last call that reads them has finished (a plan has at most one
  // call in flight): that call records tables_used on its stream.
  hipEvent_t tables_used = nullptr;
  bool tables_pending = false;

  // discrete beamforming (xeng_plan_beams): weight operands and offset terms
  int B = 0, beam_S = 0, beam_nbt = 0;
  bool beams_ready = false;
  void* d_wop = nullptr;
  int* d_bcorr = nullptr;
};

namespace {

int hip_fail(xeng_plan_t p, hipError_t e, const char* what) {
  if (p) {
    p->err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  }
  return XENG_EHIP;
}

// Create the plan's tables_used event if needed, and wait until the plan's
// last call that read its delay or weight tables has finished.
hipError_t wait_tables(xeng_plan_t p) {
  if (!p->tables_used) return hipEventCreateWithFlags(&p->tables_used, hipEventDisableTiming);
  if (!p->tables_pending) return hipSuccess;
  const hipError_t e = hipEventSynchronize(p->tables_used);
  if (e == hipSuccess) p->tables_pending = false;
  return e;
}

// After a call that read the tables: mark them in use until `s` gets here.
int mark_tables(xeng_plan_t p, hipStream_t s) {
  const hipError_t e = hipEventRecord(p->tables_used, s);
  if (e != hipSuccess) return hip_fail(p, e, "hipEventRecord");
  p->tables_pending = true;
  return XENG_OK;
}

bool flags_ok(unsigned flags, bool batch = false) {
  const unsigned form = flags & XENG_FORM_MASK;
  if (form != XENG_FORM_I8 && form != XENG_FORM_F8) return false;
  unsigned known = XENG_FORM_MASK | XENG_ACCUMULATE;
  if (batch) {
    known |= XENG_SHARED_VIS;
    if ((flags & XENG_SHARED_VIS) && !(flags & XENG_ACCUMULATE)) return false;
  }
  return (flags & ~known) == 0;
}

int ensure_cu_count(xeng_plan_t p) {
  if (p->cu_count > 0) return XENG_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(p, e, "hipGetDevice");
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(p, e, "hipDeviceGetAttribute");
  p->cu_count = cus > 0 ? cus : 1;
  return XENG_OK;
}

long long tiles_per_channel(int N) {
  const long long nt = (N + kTile - 1) / kTile;
  return nt * (nt + 1) / 2;
}

// 128 x 256 tiles (I, J) with J >= I / 2.
long long wide_tiles_per_channel(int N) {
  const long long nI = (N + kTile - 1) / kTile, nJ = (N + 2 * kTile - 1) / (2 * kTile);
  long long t = 0;
  for (long long I = 0; I < nI; ++I) t += nJ - I / 2;
  return t;
}

// Time slices per tile.  With W tiles and `slots` resident workgroups, S
// slices take round_cost(W S) rounds of 1/S of the work each; every extra
// slice costs about 4% more (exact int32 atomic adds into vis, which must be
// cleared first).  auto_slices picks the S that minimises round_cost(W S) /
// S * (1 + 0.04 (S - 1)), keeping slices of at least 1024 samples.
//
// round_cost: rounds of resident workgroups that `items` work items take on
// `slots` slots (`occupancy` per CU).  A last round that leaves each CU at
// most one workgroup costs less than a full one, since that workgroup has the
// CU to itself: on 192 tiles at N = 256 (512 slots) the timings of 1 to 8
// slices fit a cost of about 0.6 round for it.
constexpr double kLoneRound = 0.6;
double round_cost(long long items, long long slots, int occupancy) {
  const long long full = items / slots, rem = items % slots;
  if (rem == 0) return (double)full;
  return (double)full + (occupancy > 1 && rem * occupancy <= slots ? kLoneRound : 1.0);
}

double slice_cost(long long tiles, int S, long long slots, int occupancy) {
  return round_cost(tiles * S, slots, occupancy) / S * (1.0 + 0.04 * (S - 1));
}

int auto_slices(long long tiles, int T, int cu_count, int occupancy = kOccupancy) {
  const long long slots = (long long)cu_count * occupancy;
  const int smax = std::max(1, std::min(16, T / 1024));
  int best = 1;
  double best_cost = 1e300;
  for (int S = 1; S <= smax; ++S) {
    const double cost = slice_cost(tiles, S, slots, occupancy);
    if (cost < best_cost - 1e-12) {
      best_cost = cost;
      best = S;
    }
  }
  return best;
}

// Samples one launch of the 128 x 128 kernels may integrate (sums of codes
// stay exact: f32 below 2^24, int32 below 2^31).
int segment_max(int form) { return form == XENG_FORM_F8 ? XENG_F8_FLUSH_MAX : XENG_I8_SEG_MAX; }

// Time slices of a batch instance: S slices of `len` samples (a multiple of
// kChunk), from its split_t or else the batch's automatic count s_auto; no
// slice integrates more than segment_max(form) samples.
void batch_slices(const xeng_instance& d, int s_auto, int form, int& S, int& len) {
  S = d.split_t > 0 ? d.split_t : std::max(1, std::min(s_auto, d.T / 1024));
  const int seg_max = segment_max(form);
  S = std::max(S, (d.T + seg_max - 1) / seg_max);
  S = std::min(S, (d.T + kChunk - 1) / kChunk);
  len = (d.T + S - 1) / S;
  len = (len + kChunk - 1) / kChunk * kChunk;
  S = (d.T + len - 1) / len;
}

// Compute units of the current device for a plan being built; without a
// device (plans can be built and validated on a host with no GPU) the count
// of an MI355X.  Only the automatic slice count depends on it.
int cu_count_hint() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1) {
    (void)hipGetLastError();
    return 256;
  }
  return cus;
}

}  // namespace

extern "C" {

int xeng_version(void) { return (1 << 16) | 0; }

const char* xeng_strerror(int code) {
  switch (code) {
    case XENG_OK: return "success";
    case XENG_EINVAL: return "invalid argument";
    case XENG_EPLAN: return "argument does not match the plan";
    case XENG_EOVERFLOW: return "integration too long for exact int32 sums";
    case XENG_EHIP: return "HIP runtime or launch error";
    case XENG_ENOMEM: return "out of memory";
    case XENG_ELIMIT: return "request exceeds the fixed workspace of the allocation-free entry point";
    default: return "unknown error code";
  }
}

int xeng_plan(xeng_plan_t* out, int N, int F, int T_max, unsigned flags) {
  if (!out) return XENG_EINVAL;
  *out = nullptr;
  if (N < 1 || F < 1 || T_max < 1 || N > XENG_N_MAX || !flags_ok(flags)) return XENG_EINVAL;
  if (T_max > XENG_T_EXACT_MAX) return XENG_EOVERFLOW;
  xeng_plan_t p = new (std::nothrow) xeng_plan_s();
  if (!p) return XENG_ENOMEM;
  p->kind = PLAN_SINGLE;
  p->N = N;
  p->F = F;
  p->T_max = T_max;
  p->flags = flags;
  p->form = (int)(flags & XENG_FORM_MASK);
  p->accumulate = (flags & XENG_ACCUMULATE) != 0;
  *out = p;
  return XENG_OK;
}

int xeng_plan_gated(xeng_plan_t* out, int N, int F, int T_max, int G_max, unsigned flags) {
  if (!out) return XENG_EINVAL;
  *out = nullptr;
  if (G_max < 1 || G_max > XENG_G_MAX) return XENG_EINVAL;
  xeng_plan_t p = nullptr;
  int rc = xeng_plan(&p, N, F, T_max, flags);
  if (rc != XENG_OK) return rc;
  const int seg = segment_max(p->form);
  const long long nseg = (T_max + seg - 1) / seg;
  p->G_max = G_max;
  try {
    p->gate_count.assign(G_max, 0);
    p->gate_fill.assign(G_max, 0);
    p->gate_zero.assign(G_max, 0);
    p->seg_goff.assign(nseg, 0);
    p->seg_nvg.assign(nseg, 0);
  } catch (const std::bad_alloc&) {
    xeng_destroy(p);
    return XENG_ENOMEM;
  }
  // A segment has at most G_max + kSplitMax work gates (see xeng_correlate_gated).
  p->vgate_cap = nseg * ((long long)G_max + kSplitMax);
  p->gate_off_cap = p->vgate_cap + nseg;
  p->runs_cap = (long long)T_max + nseg;  // at most one run per sample, plus a cut per segment
  hipError_t e = hipHostMalloc((void**)&p->h_gate_off, p->gate_off_cap * sizeof(int),
                               hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&p->h_runs, p->runs_cap * sizeof(int2), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&p->h_vgate, p->vgate_cap * sizeof(int2), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_gate_off, p->gate_off_cap * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_runs, p->runs_cap * sizeof(int2));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_vgate, p->vgate_cap * sizeof(int2));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->gate_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    rc = e == hipErrorOutOfMemory ? XENG_ENOMEM : XENG_EHIP;
    (void)hipGetLastError();
    xeng_destroy(p);
    return rc;
  }
  *out = p;
  return XENG_OK;
}

int xeng_plan_set_delays(xeng_plan_t p, const int32_t* delays, int D_max) {
  if (!p) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE) return XENG_EPLAN;
  if (!delays) {
    p->shift = false;
    return XENG_OK;
  }
  const int N = p->N, nseg = (N + 15) / 16, nt = (N + kTile - 1) / kTile;
  if (D_max < 0 || ((long long)D_max + 64) * p->F * N >= (1LL << 31)) return XENG_EINVAL;
  std::vector<int> seg(nseg), blk(nt, 0);
  for (int n = 0; n < N; ++n) {
    if (delays[n] < 0 || delays[n] > D_max) return XENG_EINVAL;
    if (delays[n] != delays[n & ~15]) return XENG_EINVAL;  // one delay per 16-input segment
  }
  for (int k = 0; k < nseg; ++k) {
    seg[k] = delays[16 * k];
    blk[(16 * k) / kTile] = std::max(blk[(16 * k) / kTile], seg[k]);
  }
  // Uniform delays within every 128-input block are applied in the kernels'
  // loads; otherwise the frame is copied, shifted, into plan-owned memory.
  bool fine = false;
  for (int k = 0; k < nseg; ++k) fine |= seg[k] != blk[(16 * k) / kTile];
  // the plan's last call may still read the old delays
  hipError_t e = wait_tables(p);
  if (e == hipSuccess && fine && !p->d_shifted)
    e = hipMalloc((void**)&p->d_shifted, (size_t)p->T_max * p->F * N);
  if (e == hipSuccess && !p->d_seg_delay) e = hipMalloc((void**)&p->d_seg_delay, nseg * sizeof(int));
  if (e == hipSuccess && !p->d_blk_delay) e = hipMalloc((void**)&p->d_blk_delay, nt * sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_seg_delay, seg.data(), nseg * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_blk_delay, blk.data(), nt * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? XENG_ENOMEM : hip_fail(p, e, "delay upload");
  p->shift = true;
  p->shift_copy = fine;
  return XENG_OK;
}

int xeng_plan_set_tuning(xeng_plan_t p, int split_t, int kernel) {
  if (!p || split_t < 0 || kernel < 0 || kernel > 5) return XENG_EINVAL;
  p->split_t = split_t;
  p->kernel = kernel;
  return XENG_OK;
}

const char* xeng_plan_error(xeng_plan_t p) { return p ? p->err.c_str() : ""; }

// The channel kernel's slice workspace, at least `ints` int32: grown when
// needed (after the plan's last call that read it has finished), and ordered
// after that call on `s` when it may still run on another stream.
static int chan_workspace(xeng_plan_t p, size_t ints, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (!p->chan_ws_used) {
    e = hipEventCreateWithFlags(&p->chan_ws_used, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(p, e, "hipEventCreate");
  }
  if (ints > p->chan_ws_ints) {
    if (p->chan_ws_pending) {
      e = hipEventSynchronize(p->chan_ws_used);
      if (e != hipSuccess) return hip_fail(p, e, "hipEventSynchronize");
      p->chan_ws_pending = false;
    }
    if (p->d_chan_ws) (void)hipFree(p->d_chan_ws);
    p->d_chan_ws = nullptr;
    p->chan_ws_ints = 0;
    e = hipMalloc((void**)&p->d_chan_ws, ints * sizeof(int32_t));
    if (e != hipSuccess) {
      p->d_chan_ws = nullptr;
      (void)hipGetLastError();
      if (e == hipErrorOutOfMemory) return XENG_ENOMEM;
      return hip_fail(p, e, "hipMalloc (slice workspace)");
    }
    p->chan_ws_ints = ints;
  } else if (p->chan_ws_pending) {
    e = hipStreamWaitEvent(s, p->chan_ws_used, 0);
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamWaitEvent");
  }
  return XENG_OK;
}

int xeng_correlate(xeng_plan_t p, const uint8_t* samples, int N, int F, int T, int32_t* vis,
                   void* stream) {
  if (!p || !samples || !vis || N < 1 || F < 1 || T < 1) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE) return XENG_EPLAN;
  if (T > XENG_T_EXACT_MAX) return XENG_EOVERFLOW;
  if (N != p->N || F != p->F || T > p->T_max) return XENG_EPLAN;
  int rc = ensure_cu_count(p);
  if (rc != XENG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // delays: in the loads, or by a shifted copy of the frame
  const bool kshift = p->shift && !p->shift_copy;
  if (p->shift && p->shift_copy) {
    hipError_t e = xeng::launch_shift_copy(samples, p->d_shifted, N, F, T, p->d_seg_delay, s);
    if (e != hipSuccess) return hip_fail(p, e, "shift copy launch");
    samples = p->d_shifted;
  }

  const int nt = (N + kTile - 1) / kTile;
  // fast loads: 16-byte row pieces, and per-lane offsets that fit 32 bits
  const bool aligned = (N % 16 == 0) && ((reinterpret_cast<uintptr_t>(samples) & 15) == 0) &&
                       ((long long)F * N <= (1LL << 25));
  // wide tiles (128 x 256, one workgroup per CU) only on request and when
  // the rows allow fast loads; 128 x 128 (two workgroups per CU) otherwise
  const bool wide = aligned && p->kernel == 2 && !kshift;
  // the channel kernel (int8, N <= 256): on request, or automatically above
  // one tile edge when the rows allow fast loads
  const bool chan = p->form == XENG_FORM_I8 && !kshift && N <= kChanMax &&
                    (p->kernel == 5 || (p->kernel == 0 && N > kTile && aligned));
  const long long tpc = wide ? wide_tiles_per_channel(N) : tiles_per_channel(N);
  const int occupancy = wide ? 1 : kOccupancy;
  // The FP8 form integrates at most XENG_F8_FLUSH_MAX samples per launch (f32
  // sums of codes stay exact below 2^24), the int8 form on 128 x 128 tiles at
  // most XENG_I8_SEG_MAX (int32 sums of codes below 2^31); later launches add
  // their sums in stream order.  The wide int8 kernel does the whole frame in
  // one launch.
  const int seg = p->form == XENG_FORM_F8 ? XENG_F8_FLUSH_MAX : (wide ? T : XENG_I8_SEG_MAX);
  for (int t0 = 0; t0 < T; t0 += seg) {
    const int t1 = std::min(T, t0 + seg), len = t1 - t0;
    if (chan) {
      // one work item per (channel, slice), one workgroup per CU
      int ns = p->split_t > 0 ? p->split_t : auto_slices(F, len, p->cu_count, 1);
      ns = std::min(ns, (len + kChunk - 1) / kChunk);
      int sl = (len + ns - 1) / ns;
      sl = (sl + kChunk - 1) / kChunk * kChunk;
      ns = (len + sl - 1) / sl;
      const bool add = p->accumulate || t0 > 0;
      const long long part = (long long)F * N * (N + 1);  // ints of one slice's triangles
      if (ns > 1) {
        rc = chan_workspace(p, (size_t)ns * (size_t)part, s);
        if (rc != XENG_OK) return rc;
      }
      xeng::ChanArgs c;
      c.samples = samples;
      c.vis = vis;
      c.N = N;
      c.F = F;
      c.t0 = t0;
      c.t1 = t1;
      c.nslices = ns;
      c.slice_len = sl;
      c.row_stride = (long long)F * N;
      // one slice writes vis itself; several store their own triangles into
      // the workspace, and a second kernel sums them into vis
      c.partial = ns > 1 ? p->d_chan_ws : nullptr;
      c.write_mode = (ns == 1 && add) ? xeng::WM_ADD : xeng::WM_STORE;
      hipError_t e = xeng::launch_chan(c, aligned, s);
      if (e != hipSuccess) return hip_fail(p, e, "channel kernel launch");
      if (ns > 1) {
        e = xeng::launch_chan_reduce(p->d_chan_ws, vis, part, ns, add, s);
        if (e != hipSuccess) return hip_fail(p, e, "slice sum launch");
        e = hipEventRecord(p->chan_ws_used, s);
        if (e != hipSuccess) return hip_fail(p, e, "hipEventRecord");
        p->chan_ws_pending = true;
      }
      continue;
    }
    const long long W = tpc * F;  // tiles of the launch
    int nslices = p->split_t > 0 ? p->split_t : auto_slices(W, len, p->cu_count, occupancy);
    nslices = std::min(nslices, (len + kChunk - 1) / kChunk);
    int slice_len = (len + nslices - 1) / nslices;
    slice_len = (slice_len + kChunk - 1) / kChunk * kChunk;
    nslices = (len + slice_len - 1) / slice_len;
    const bool add = p->accumulate || t0 > 0;

    // Automatic choice between uniform slices and a head/tail split: R full
    // rounds of whole tiles (plain stores or adds), then the remaining tiles
    // cut into S_t slices that fill one more round (atomic adds into a
    // cleared region).  Same cost model as auto_slices.
    const long long slots = (long long)p->cu_count * occupancy;
    long long head = W;
    int tail_slices = 0, tail_len = 0;
    if (p->split_t == 0 && !wide && W > slots && W % slots != 0 && slots % 8 == 0) {
      const long long R = W / slots, rem = W - R * slots;
      const int smax = std::max(1, std::min(16, len / 1024));
      int St = (int)std::min<long long>(smax, std::max<long long>(1, (slots + rem / 2) / rem));
      int tl = (len + St - 1) / St;
      tl = (tl + kChunk - 1) / kChunk * kChunk;
      St = (len + tl - 1) / tl;
      const double cost_tail = (double)R + slice_cost(rem, St, slots, occupancy);
      if (St > 1 && cost_tail < slice_cost(W, nslices, slots, occupancy) - 1e-9) {
        head = R * slots;
        tail_slices = St;
        tail_len = tl;
        nslices = 1;
        slice_len = len;
      }
    }

    xeng::TileArgs a;
    a.samples = samples;
    a.vis = vis;
    a.N = N;
    a.F = F;
    a.t0 = t0;
    a.t1 = t1;
    a.nt = nt;
    a.tiles_per_chan = (int)tpc;
    a.nslices = nslices;
    a.slice_len = slice_len;
    a.row_stride = (long long)F * N;
    a.head_tiles = (int)head;
    a.tail_slices = tail_slices;
    a.tail_len = tail_len;
    a.tail_mode = xeng::WM_ATOMIC;
    // Diagonal tiles split the sub-tile above the diagonal between two waves
    // where they are a large share of the tiles (N <= 1024: at least 2 in 9);
    // at N = 2048 (16 in 136) the uniform tile time of the common roles pays
    // more (measured on the full-array frame).
    a.split_diag = p->kernel == 3 ? 1 : p->kernel == 4 ? 0 : (nt <= 8 ? 1 : 0);
    a.seg_delay = kshift ? p->d_seg_delay : nullptr;
    a.blk_delay = kshift ? p->d_blk_delay : nullptr;
    if (nslices > 1) {
      a.write_mode = xeng::WM_ATOMIC;
      if (!add) {
        hipError_t e = xeng::launch_zero(vis, (long long)F * N * (N + 1), s);
        if (e != hipSuccess) return hip_fail(p, e, "zero fill launch");
      }
    } else {
      a.write_mode = add ? xeng::WM_ADD : xeng::WM_STORE;
    }
    if (tail_slices > 0 && !add) {
      hipError_t e = xeng::launch_zero_tiles(vis, N, (int)tpc, nt, (int)head, (int)(W - head), s);
      if (e != hipSuccess) return hip_fail(p, e, "tail zero launch");
    }
    hipError_t e = wide ? xeng::launch_wide(a, p->form, s) : xeng::launch_tiles(a, p->form, aligned, s);
    if (e != hipSuccess) return hip_fail(p, e, "correlation kernel launch");
  }
  return p->shift ? mark_tables(p, s) : XENG_OK;
}

int xeng_correlate_gated(xeng_plan_t p, const uint8_t* samples, int N, int F, int T,
                         const int32_t* gate, int G, int32_t* vis, void* stream) {
  if (!p || !samples || !gate || !vis || N < 1 || F < 1 || T < 1 || G < 1) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE || p->G_max < 1 || G > p->G_max) return XENG_EPLAN;
  if (T > XENG_T_EXACT_MAX) return XENG_EOVERFLOW;
  if (N != p->N || F != p->F || T > p->T_max) return XENG_EPLAN;
  int rc = ensure_cu_count(p);
  if (rc != XENG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->gate_pending) {
    // the pinned staging may still be read by the previous call's copy
    hipError_t e = hipEventSynchronize(p->gate_done);
    if (e != hipSuccess) return hip_fail(p, e, "hipEventSynchronize");
    p->gate_pending = false;
  }
  // Runs of equal gate per launch segment, grouped by gate in time order,
  // then cut into work gates.  A run is integrated in whole chunks of kChunk
  // samples, and the sums of codes are exact only while a work item
  // integrates at most `seg` chunk-rounded samples.  Runs of 64 samples or
  // more never exceed that (a segment holds at most `seg` samples), but a gate
  // with many shorter runs can: its runs are then split, greedily in time
  // order, into groups that fit, each its own work gate adding into the
  // gate's buffer with int32 atomics (cleared first when the call
  // overwrites).  Two consecutive groups of a gate hold more than `seg`
  // chunk-rounded samples, and a segment holds at most 64 seg of them, so a
  // segment has fewer than kSplitMax extra work gates.
  const int seg = segment_max(p->form);
  const int nseg = (T + seg - 1) / seg;
  long long nruns = 0, ngoff = 0, nvg = 0;
  int* count = p->gate_count.data();
  int* fill = p->gate_fill.data();
  int* zero = p->gate_zero.data();
  std::fill(zero, zero + G, 0);
  for (int k = 0; k < nseg; ++k) {
    const int t0 = k * seg, t1 = std::min(T, t0 + seg);
    const int mode = (p->accumulate || k > 0) ? xeng::WM_ADD : xeng::WM_STORE;
    std::fill(count, count + G, 0);
    for (int t = t0; t < t1;) {  // count the runs of each gate
      const int g = gate[t];
      int u = t + 1;
      while (u < t1 && gate[u] == g) ++u;
      if (g >= 0 && g < G) ++count[g];
      t = u;
    }
    fill[0] = (int)nruns;
    for (int g = 1; g < G; ++g) fill[g] = fill[g - 1] + count[g - 1];
    for (int t = t0; t < t1;) {  // place them, in time order per gate
      const int g = gate[t];
      int u = t + 1;
      while (u < t1 && gate[u] == g) ++u;
      if (g >= 0 && g < G) p->h_runs[fill[g]++] = make_int2(t, u);
      t = u;
    }
    // work gates: fill[g] now ends gate g's runs
    p->seg_goff[k] = (int)ngoff;
    const long long vg0 = nvg;
    int r = (int)nruns;
    for (int g = 0; g < G; ++g) {
      const int r_end = fill[g];
      const long long first = nvg;
      int b = r;
      long long padded = 0;
      for (int e = r; e < r_end; ++e) {
        const int2 run = p->h_runs[e];
        const long long pl = (long long)(run.y - run.x + kChunk - 1) / kChunk * kChunk;
        if (e > b && padded + pl > seg) {
          p->h_gate_off[ngoff++] = b;
          p->h_vgate[nvg++] = make_int2(g, xeng::WM_ATOMIC);
          b = e;
          padded = 0;
        }
        padded += pl;
      }
      const bool split = nvg > first;
      p->h_gate_off[ngoff++] = b;
      p->h_vgate[nvg++] = make_int2(g, split ? xeng::WM_ATOMIC : mode);
      if (split && mode == xeng::WM_STORE) zero[g] = 1;
      r = r_end;
    }
    p->h_gate_off[ngoff++] = r;
    nruns = r;
    p->seg_nvg[k] = (int)(nvg - vg0);
  }
  hipError_t e = hipSuccess;
  if (nruns > 0)
    e = hipMemcpyAsync(p->d_runs, p->h_runs, nruns * sizeof(int2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_gate_off, p->h_gate_off, (size_t)ngoff * sizeof(int),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_vgate, p->h_vgate, (size_t)nvg * sizeof(int2), hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess) e = hipEventRecord(p->gate_done, s);
  if (e != hipSuccess) return hip_fail(p, e, "gate table upload");
  p->gate_pending = true;

  const bool kshift = p->shift && !p->shift_copy;
  if (p->shift && p->shift_copy) {
    e = xeng::launch_shift_copy(samples, p->d_shifted, N, F, T, p->d_seg_delay, s);
    if (e != hipSuccess) return hip_fail(p, e, "shift copy launch");
    samples = p->d_shifted;
  }
  const bool aligned = (N % 16 == 0) && ((reinterpret_cast<uintptr_t>(samples) & 15) == 0) &&
                       ((long long)F * N <= (1LL << 25));
  // split gates that overwrite: their buffers are cleared first (the buffers
  // of consecutive gates are contiguous in the gate-major output)
  const long long gate_words = (long long)F * N * (N + 1);
  for (int g = 0; g < G;) {
    if (!zero[g]) {
      ++g;
      continue;
    }
    int h = g;
    while (h < G && zero[h]) ++h;
    e = xeng::launch_zero(vis + g * gate_words, (h - g) * gate_words, s);
    if (e != hipSuccess) return hip_fail(p, e, "gate clear launch");
    g = h;
  }
  for (int k = 0; k < nseg; ++k) {
    xeng::GatedArgs a;
    a.samples = samples;
    a.vis = vis;
    a.N = N;
    a.F = F;
    a.G = p->seg_nvg[k];
    a.nt = (N + kTile - 1) / kTile;
    a.tiles_per_chan = (int)tiles_per_channel(N);
    a.write_mode = (p->accumulate || k > 0) ? xeng::WM_ADD : xeng::WM_STORE;
    a.gate_off = p->d_gate_off + p->seg_goff[k];
    a.runs = p->d_runs;
    a.vgate = p->d_vgate + (p->seg_goff[k] - k);
    a.row_stride = (long long)F * N;
    a.seg_delay = kshift ? p->d_seg_delay : nullptr;
    a.blk_delay = kshift ? p->d_blk_delay : nullptr;
    // adding: a work gate without runs adds nothing
    a.skip_empty = a.write_mode == xeng::WM_ADD ? 1 : 0;
    e = xeng::launch_gated(a, p->form, aligned, s);
    if (e != hipSuccess) return hip_fail(p, e, "gated correlation kernel launch");
  }
  return p->shift ? mark_tables(p, s) : XENG_OK;
}

// Event rows a frame of T samples can need per channel: a block of rows never
// takes more event rows than it has rows with several invalid inputs.
static long long flag_rows(int T) { return T; }

int xeng_plan_flagged(xeng_plan_t* out, int N, int F, int T_max, unsigned flags) {
  if (!out) return XENG_EINVAL;
  *out = nullptr;
  xeng_plan_t p = nullptr;
  int rc = xeng_plan(&p, N, F, T_max, flags);
  if (rc != XENG_OK) return rc;
  p->flagged = true;
  p->flag_cap = flag_rows(T_max);
  p->flag_nseg = (int)((p->flag_cap + XENG_I8_SEG_MAX - 1) / XENG_I8_SEG_MAX);
  const long long NB = (long long)N * (N + 1) / 2;
  const long long nint = (long long)F + 2LL * F * N + 1 + 2LL * p->flag_nseg;
  hipError_t e = hipMalloc((void**)&p->d_fU, (size_t)(p->flag_cap * F * N));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_fX, (size_t)(F * NB * 2) * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_fint, (size_t)nint * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_fruns, (size_t)p->flag_nseg * sizeof(int2));
  if (e != hipSuccess) {
    rc = e == hipErrorOutOfMemory ? XENG_ENOMEM : XENG_EHIP;
    (void)hipGetLastError();
    xeng_destroy(p);
    return rc;
  }
  *out = p;
  return XENG_OK;
}

int xeng_correlate_flagged(xeng_plan_t p, uint8_t* samples, const uint32_t* flags, int N, int F,
                           int T, int32_t* vis, int32_t* counts, void* stream) {
  if (!p || !samples || !flags || !vis || !counts || N < 1 || F < 1 || T < 1) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE || !p->flagged || p->shift) return XENG_EPLAN;
  if (T > XENG_T_EXACT_MAX) return XENG_EOVERFLOW;
  if (N != p->N || F != p->F || T > p->T_max) return XENG_EPLAN;
  hipStream_t s = static_cast<hipStream_t>(stream);
  xeng::FlagArgs a;
  a.samples = samples;
  a.flags = flags;
  a.N = N;
  a.F = F;
  a.T = T;
  a.W = (N + 31) / 32;
  a.U = p->d_fU;
  a.cap = flag_rows(T);
  a.cnt = p->d_fint;
  a.single = a.cnt + F;
  a.n = a.single + (long long)F * N;
  a.R = a.n + (long long)F * N;
  a.fgate_off = a.R + 1;
  a.X = p->d_fX;
  a.fruns = p->d_fruns;
  a.counts = counts;
  const int nseg = (int)((a.cap + XENG_I8_SEG_MAX - 1) / XENG_I8_SEG_MAX);
  hipError_t e = xeng::launch_flag_scan(a, nseg, XENG_I8_SEG_MAX, s);
  if (e != hipSuccess) return hip_fail(p, e, "flag scan launch");
  // the frame, now with every flagged sample zero
  int rc = xeng_correlate(p, samples, N, F, T, vis, stream);
  if (rc != XENG_OK) return rc;
  // the event rows: Re X_ij = rows where i and j are both invalid
  const bool aligned = (N % 16 == 0) && ((long long)F * N <= (1LL << 25));
  for (int k = 0; k < nseg; ++k) {
    xeng::GatedArgs g;
    g.samples = p->d_fU;
    g.vis = p->d_fX;
    g.N = N;
    g.F = F;
    g.G = 1;
    g.nt = (N + kTile - 1) / kTile;
    g.tiles_per_chan = (int)tiles_per_channel(N);
    g.write_mode = k > 0 ? xeng::WM_ADD : xeng::WM_STORE;
    g.gate_off = a.fgate_off + 2 * k;
    g.runs = p->d_fruns;
    g.row_stride = (long long)F * N;
    g.seg_delay = nullptr;
    g.blk_delay = nullptr;
    g.vgate = nullptr;
    g.skip_empty = 1;
    e = xeng::launch_gated(g, XENG_FORM_I8, aligned, s);
    if (e != hipSuccess) return hip_fail(p, e, "event correlation kernel launch");
  }
  e = xeng::launch_flag_counts(a, p->accumulate ? 1 : 0, s);
  if (e != hipSuccess) return hip_fail(p, e, "flag count launch");
  return XENG_OK;
}

int xeng_normalize(xeng_plan_t p, const int32_t* vis, const int32_t* counts, double scale,
                   float* out, void* stream) {
  if (!p || !vis || !counts || !out || !(scale > 0.0) || !(scale < 1e300)) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE) return XENG_EPLAN;
  const long long n = (long long)p->F * p->N * (p->N + 1) / 2;
  hipError_t e = xeng::launch_normalize(vis, counts, n, scale, out,
                                        static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(p, e, "normalize launch");
  return XENG_OK;
}

// Beamforming launches: a launch of T rows reads at byte offsets below
// (T + 512) F N + N + 160 from its first row (more than the rows of one
// workgroup past the frame, plus a step past the row), which the segment
// length keeps below 2^31.
constexpr long long kBeamRowsMax = 512;
long long beam_segment(long long row) { return ((1LL << 31) - 1 - 256) / row - kBeamRowsMax - 2; }

int xeng_plan_beams(xeng_plan_t* out, int N, int F, int T_max, int B, unsigned flags) {
  if (!out) return XENG_EINVAL;
  *out = nullptr;
  if (flags != 0 || B < 1 || B > XENG_BEAMS_MAX) return XENG_EINVAL;
  if (N < 1 || F < 1 || N > XENG_N_MAX || beam_segment((long long)F * N) < 1) return XENG_EINVAL;
  xeng_plan_t p = nullptr;
  int rc = xeng_plan(&p, N, F, T_max, 0);
  if (rc != XENG_OK) return rc;
  p->B = B;
  p->beam_S = (N + 127) / 128;
  p->beam_nbt = (2 * B + 31) / 32;
  const size_t wop_bytes = (size_t)F * p->beam_S * 8 * p->beam_nbt * 64 * 16;
  hipError_t e = hipMalloc(&p->d_wop, wop_bytes);
  if (e == hipSuccess)
    e = hipMalloc((void**)&p->d_bcorr, (size_t)F * p->beam_nbt * 32 * sizeof(int));
  if (e != hipSuccess) {
    rc = e == hipErrorOutOfMemory ? XENG_ENOMEM : XENG_EHIP;
    (void)hipGetLastError();
    xeng_destroy(p);
    return rc;
  }
  *out = p;
  return XENG_OK;
}

int xeng_beam_set_weights(xeng_plan_t p, const int8_t* weights) {
  if (!p || !weights) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE || p->B < 1) return XENG_EPLAN;
  const int N = p->N, F = p->F, B = p->B, S = p->beam_S, NBT = p->beam_nbt;
  const long long nw = (long long)F * B * N * 2;
  for (long long e = 0; e < nw; ++e)
    if (weights[e] == -128) return XENG_EINVAL;  // -w must be an int8 as well
  // Operand of (f, step s, k-step q, tile c, lane l): bytes e = 0..7 weigh the
  // real code of input 128 s + 32 (q >> 1) + 16 (l >> 5) + 8 (q & 1) + e,
  // bytes 8 + e its imaginary code, for column 32 c + (l & 31) = 2 b + comp of
  // the real contraction: comp 0 (Re y) takes (w_re, -w_im), comp 1 (Im y)
  // (w_im, w_re).
  std::vector<int8_t> wop((size_t)F * S * 8 * NBT * 64 * 16, 0);
  std::vector<int> corr((size_t)F * NBT * 32, 0);
  for (int f = 0; f < F; ++f)
    for (int s = 0; s < S; ++s)
      for (int q = 0; q < 8; ++q)
        for (int c = 0; c < NBT; ++c)
          for (int l = 0; l < 64; ++l) {
            const int col = 32 * c + (l & 31), b = col >> 1, comp = col & 1;
            if (b >= B) continue;
            int8_t* o = &wop[(((((size_t)f * S + s) * 8 + q) * NBT + c) * 64 + l) * 16];
            for (int e = 0; e < 8; ++e) {
              const int n = 128 * s + 32 * (q >> 1) + 16 * (l >> 5) + 8 * (q & 1) + e;
              if (n >= N) continue;
              const int8_t* w = weights + (((size_t)f * B + b) * N + n) * 2;
              const int cr = comp == 0 ? w[0] : w[1];
              const int ci = comp == 0 ? -w[1] : w[0];
              o[e] = (int8_t)cr;
              o[8 + e] = (int8_t)ci;
              corr[(size_t)f * NBT * 32 + col] += 8 * (cr + ci);
            }
          }
  // the plan's last call may still read the old operands
  hipError_t e = wait_tables(p);
  if (e == hipSuccess) e = hipMemcpy(p->d_wop, wop.data(), wop.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_bcorr, corr.data(), corr.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(p, e, "beam weight upload");
  p->beams_ready = true;
  return XENG_OK;
}

int xeng_beamform(xeng_plan_t p, const uint8_t* samples, int N, int F, int T, int32_t* beams,
                  void* stream) {
  if (!p || !samples || !beams || N < 1 || F < 1 || T < 1) return XENG_EINVAL;
  if (p->kind != PLAN_SINGLE || p->B < 1 || !p->beams_ready) return XENG_EPLAN;
  if (N != p->N || F != p->F || T > p->T_max) return XENG_EPLAN;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long row = (long long)F * N;
  const long long seg = beam_segment(row);  // >= 1 by the plan's check
  const bool aligned = (N % 16 == 0) && ((reinterpret_cast<uintptr_t>(samples) & 15) == 0);
  for (long long t0 = 0; t0 < T; t0 += seg) {
    xeng::BeamArgs a;
    a.samples = samples + t0 * row;
    a.beams = beams + t0 * F * 2LL * p->B;
    a.wop = p->d_wop;
    a.corr = p->d_bcorr;
    a.N = N;
    a.F = F;
    a.T = (int)std::min<long long>(seg, T - t0);
    a.B = p->B;
    a.S = p->beam_S;
    a.NBT = p->beam_nbt;
    a.tblocks = 0;
    for (int c0 = 0; c0 < p->beam_nbt; c0 += 4) {
      a.c0 = c0;
      const hipError_t e = xeng::launch_beams(a, std::min(4, p->beam_nbt - c0), aligned, s);
      if (e != hipSuccess) return hip_fail(p, e, "beamform kernel launch");
    }
  }
  return mark_tables(p, s);
}

int xeng_plan_batch(xeng_plan_t* out, const xeng_instance* descs, int count, unsigned flags) {
  if (!out) return XENG_EINVAL;
  *out = nullptr;
  if (!descs || count < 1 || !flags_ok(flags, true)) return XENG_EINVAL;
  for (int k = 0; k < count; ++k) {
    const xeng_instance& d = descs[k];
    if (d.N < 1 || d.F < 1 || d.T < 1 || d.N > XENG_N_MAX || d.split_t < 0) return XENG_EINVAL;
  }
  for (int k = 0; k < count; ++k)
    if (descs[k].T > XENG_T_EXACT_MAX) return XENG_EOVERFLOW;
  xeng_plan_t p = new (std::nothrow) xeng_plan_s();
  if (!p) return XENG_ENOMEM;
  p->kind = PLAN_BATCH;
  p->flags = flags;
  p->form = (int)(flags & XENG_FORM_MASK);
  p->accumulate = (flags & XENG_ACCUMULATE) != 0;
  const bool shared = (flags & XENG_SHARED_VIS) != 0;
  try {
    p->insts.assign(descs, descs + count);
    p->inst_zero.assign(count, 0);
    struct Costed {
      long long cost;
      xeng::BatchItem it;
    };
    std::vector<Costed> work;
    // automatic slices (split_t = 0): one count for the whole batch, from its
    // total tiles, so that a launch of few instances still fills the GPU
    long long batch_tiles = 0;
    for (int k = 0; k < count; ++k) batch_tiles += descs[k].F * tiles_per_channel(descs[k].N);
    const int s_auto = auto_slices(batch_tiles, XENG_T_EXACT_MAX, cu_count_hint());
    for (int k = 0; k < count; ++k) {
      const xeng_instance& d = descs[k];
      const int nt = (d.N + kTile - 1) / kTile;
      int S = 0, len = 0;
      batch_slices(d, s_auto, p->form, S, len);
      const int mode = (S > 1 || shared) ? xeng::WM_ATOMIC
                                         : (p->accumulate ? xeng::WM_ADD : xeng::WM_STORE);
      if (S > 1 && !p->accumulate) {
        p->inst_zero[k] = 1;
        p->any_zero = true;
      }
      for (int f = 0; f < d.F; ++f)
        for (int I = 0; I < nt; ++I)
          for (int J = I; J < nt; ++J)
            for (int s = 0; s < S; ++s) {
              xeng::BatchItem it;
              it.inst = k;
              it.f = f;
              it.I = I;
              it.J = J;
              it.t0 = s * len;
              it.t1 = std::min(d.T, (s + 1) * len);
              it.mode = mode;
              it.pad = 0;
              // cost: MFMA blocks that hold baselines x samples
              const int rows = std::min(kTile, d.N - I * kTile);
              const int cols = std::min(kTile, d.N - J * kTile);
              long long area = I == J ? (long long)rows * (rows + 1) / 2 : (long long)rows * cols;
              work.push_back({area * (it.t1 - it.t0), it});
            }
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const Costed& x, const Costed& y) { return x.cost > y.cost; });
    p->items.reserve(work.size());
    for (const Costed& c : work) p->items.push_back(c.it);
  } catch (const std::bad_alloc&) {
    delete p;
    return XENG_ENOMEM;
  }
  if (p->items.size() > 0x7fffffffu) {
    delete p;
    return XENG_EINVAL;
  }
  *out = p;
  return XENG_OK;
}

static int batch_setup(xeng_plan_t p) {
  if (p->d_items) return XENG_OK;
  int rc = ensure_cu_count(p);
  if (rc != XENG_OK) return rc;
  const size_t ni = p->insts.size(), nw = p->items.size();
  hipError_t e = hipHostMalloc((void**)&p->h_insts, kStageRing * ni * sizeof(xeng::BatchInst),
                               hipHostMallocDefault);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? XENG_ENOMEM : hip_fail(p, e, "hipHostMalloc");
  e = hipMalloc((void**)&p->d_insts, ni * sizeof(xeng::BatchInst));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_items, nw * sizeof(xeng::BatchItem));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_counter, sizeof(int));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? XENG_ENOMEM : hip_fail(p, e, "hipMalloc");
  e = hipMemcpy(p->d_items, p->items.data(), nw * sizeof(xeng::BatchItem), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(p, e, "work list upload");
  for (int r = 0; r < kStageRing && e == hipSuccess; ++r)
    e = hipEventCreateWithFlags(&p->copy_done[r], hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(p, e, "hipEventCreate");
  return XENG_OK;
}

// Bring the device instance table up to date with these pointers (a no-op
// when they are the ones already uploaded).
static int batch_upload(xeng_plan_t p, const uint8_t* const* samples, int32_t* const* vis,
                        hipStream_t s) {
  const size_t ni = p->insts.size();
  bool same = p->uploaded.size() == 2 * ni;
  for (size_t k = 0; same && k < ni; ++k)
    same = p->uploaded[2 * k] == samples[k] &&
           p->uploaded[2 * k + 1] == (samples[k] ? vis[k] : nullptr);
  if (same) return XENG_OK;
  const int r = p->stage_next;
  p->stage_next = (r + 1) % kStageRing;
  if (p->copy_pending[r]) {
    // this staging copy may still be read by an earlier call's upload
    hipError_t e = hipEventSynchronize(p->copy_done[r]);
    if (e != hipSuccess) return hip_fail(p, e, "hipEventSynchronize");
    p->copy_pending[r] = false;
  }
  xeng::BatchInst* stage = p->h_insts + (size_t)r * ni;
  p->uploaded.assign(2 * ni, nullptr);
  for (size_t k = 0; k < ni; ++k) {
    const xeng_instance& d = p->insts[k];
    xeng::BatchInst& b = stage[k];
    b.samples = samples[k];
    b.vis = samples[k] ? vis[k] : nullptr;
    b.N = d.N;
    b.F = d.F;
    b.T = d.T;
    b.aligned = (d.N % 16 == 0) && ((reinterpret_cast<uintptr_t>(samples[k]) & 15) == 0) &&
                ((long long)d.F * d.N <= (1LL << 25));
    b.zero = samples[k] ? p->inst_zero[k] : 0;
    b.pad = 0;
    p->uploaded[2 * k] = samples[k];
    p->uploaded[2 * k + 1] = b.vis;
  }
  hipError_t e = hipMemcpyAsync(p->d_insts, stage, ni * sizeof(xeng::BatchInst),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(p->copy_done[r], s);
  if (e != hipSuccess) {
    p->uploaded.clear();
    return hip_fail(p, e, "instance table upload");
  }
  p->copy_pending[r] = true;
  return XENG_OK;
}

static int batch_check(xeng_plan_t p, const uint8_t* const* samples, int32_t* const* vis) {
  if (!p || !samples || !vis) return XENG_EINVAL;
  if (p->kind != PLAN_BATCH) return XENG_EPLAN;
  for (size_t k = 0; k < p->insts.size(); ++k)
    if (samples[k] && !vis[k]) return XENG_EINVAL;
  return XENG_OK;
}

static int batch_grid(xeng_plan_t p) {
  const long long g = std::min<long long>((long long)p->cu_count * kOccupancy,
                                          (long long)p->items.size());
  return (int)std::max(1LL, g);
}

int xeng_correlate_batch(xeng_plan_t p, const uint8_t* const* samples, int32_t* const* vis,
                         void* stream) {
  int rc = batch_check(p, samples, vis);
  if (rc != XENG_OK) return rc;
  rc = batch_setup(p);
  if (rc != XENG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = batch_upload(p, samples, vis, s);
  if (rc != XENG_OK) return rc;
  hipError_t e = xeng::launch_batch(p->d_insts, (int)p->insts.size(), p->d_items,
                                    (int)p->items.size(), p->d_counter, batch_grid(p), p->form,
                                    p->any_zero, s);
  if (e != hipSuccess) return hip_fail(p, e, "batch kernel launch");
  return XENG_OK;
}

int xeng_correlate_batch_graph(xeng_plan_t p, const uint8_t* const* samples,
                               int32_t* const* vis, void* stream) {
  int rc = batch_check(p, samples, vis);
  if (rc != XENG_OK) return rc;
  rc = batch_setup(p);
  if (rc != XENG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = batch_upload(p, samples, vis, s);
  if (rc != XENG_OK) return rc;
  if (!p->graph_exec) {
    // The kernels read every pointer from the device instance table, so one
    // captured graph serves every set of buffers.
    hipError_t e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamCreate");
    e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamBeginCapture");
    hipError_t le = xeng::launch_batch(p->d_insts, (int)p->insts.size(), p->d_items,
                                       (int)p->items.size(), p->d_counter, batch_grid(p),
                                       p->form, p->any_zero, p->capture_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->capture_stream, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(p, le, "batch kernel capture");
    }
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->graph_exec = nullptr;
      return hip_fail(p, e, "hipGraphInstantiate");
    }
  }
  hipError_t e = hipGraphLaunch(p->graph_exec, s);
  if (e != hipSuccess) return hip_fail(p, e, "hipGraphLaunch");
  return XENG_OK;
}

int xeng_correlate_batch_noalloc(const xeng_instance* descs, int count, unsigned flags,
                                 const uint8_t* const* samples, int32_t* const* vis,
                                 void* stream) {
  if (!descs || !samples || !vis || count < 1 || !flags_ok(flags, true)) return XENG_EINVAL;
  int active = 0;
  for (int k = 0; k < count; ++k) {
    const xeng_instance& d = descs[k];
    if (d.N < 1 || d.F < 1 || d.T < 1 || d.N > XENG_N_MAX || d.split_t < 0) return XENG_EINVAL;
    if (samples[k] && !vis[k]) return XENG_EINVAL;
    active += samples[k] ? 1 : 0;
  }
  for (int k = 0; k < count; ++k)
    if (descs[k].T > XENG_T_EXACT_MAX) return XENG_EOVERFLOW;
  if (active > XENG_NOALLOC_INST_MAX) return XENG_ELIMIT;
  // every tile takes at least one work item
  long long tiles = 0;
  for (int k = 0; k < count; ++k)
    if (samples[k]) tiles += descs[k].F * tiles_per_channel(descs[k].N);
  if (tiles > XENG_NOALLOC_ITEMS_MAX) return XENG_ELIMIT;
  if (active == 0) return XENG_OK;

  unsigned char* ws = nullptr;
  int cus = 0;
  if (xeng::noalloc_workspace(&ws, &cus) != hipSuccess) {
    (void)hipGetLastError();
    return XENG_EHIP;
  }
  const int form = (int)(flags & XENG_FORM_MASK);
  const bool accumulate = (flags & XENG_ACCUMULATE) != 0;
  const bool shared = (flags & XENG_SHARED_VIS) != 0;
  // the same schedule rules as xeng_plan_batch, over the active instances;
  // instances go in decreasing order of their largest work item, so that
  // the longest items start first
  const int s_auto = auto_slices(tiles, XENG_T_EXACT_MAX, cus);
  xeng::NoallocArgs a;
  long long cost[XENG_NOALLOC_INST_MAX];
  int order[XENG_NOALLOC_INST_MAX];
  int n = 0;
  long long nitems = 0;
  bool any_zero = false;
  for (int k = 0; k < count; ++k) {
    if (!samples[k]) continue;
    const xeng_instance& d = descs[k];
    xeng::NoallocInst& in = a.inst[n];
    int S = 0, len = 0;
    batch_slices(d, s_auto, form, S, len);
    const int mode = (S > 1 || shared) ? xeng::WM_ATOMIC
                                       : (accumulate ? xeng::WM_ADD : xeng::WM_STORE);
    const bool zero = S > 1 && !accumulate;
    const bool aligned = (d.N % 16 == 0) && ((reinterpret_cast<uintptr_t>(samples[k]) & 15) == 0) &&
                         ((long long)d.F * d.N <= (1LL << 25));
    in.samples = samples[k];
    in.vis = vis[k];
    in.N = d.N;
    in.F = d.F;
    in.T = d.T;
    in.S = S;
    in.len = len;
    in.flags = mode | (zero ? 4 : 0) | (aligned ? 8 : 0);
    in.first = 0;
    in.pad = 0;
    any_zero |= zero;
    nitems += (long long)d.F * tiles_per_channel(d.N) * S;
    const long long edge = std::min(kTile, d.N);
    cost[n] = edge * edge * len;
    order[n] = n;
    ++n;
  }
  if (nitems > XENG_NOALLOC_ITEMS_MAX) return XENG_ELIMIT;
  for (int i = 1; i < n; ++i)  // insertion sort by decreasing cost (stable)
    for (int j = i; j > 0 && cost[order[j]] > cost[order[j - 1]]; --j)
      std::swap(order[j], order[j - 1]);
  xeng::NoallocInst sorted[XENG_NOALLOC_INST_MAX];
  int first = 0;
  for (int i = 0; i < n; ++i) {
    sorted[i] = a.inst[order[i]];
    sorted[i].first = first;
    first += sorted[i].F * (int)tiles_per_channel(sorted[i].N) * sorted[i].S;
  }
  std::copy(sorted, sorted + n, a.inst);
  a.ws = ws;
  a.ninst = n;
  a.nitems = (int)nitems;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = xeng::launch_noalloc_prep(a, s);
  if (e == hipSuccess) {
    const int grid = (int)std::max(1LL, std::min<long long>((long long)cus * kOccupancy, nitems));
    e = xeng::launch_batch(reinterpret_cast<const xeng::BatchInst*>(ws + xeng::kNoallocInstOff),
                           n, reinterpret_cast<const xeng::BatchItem*>(ws + xeng::kNoallocItemsOff),
                           (int)nitems, reinterpret_cast<int*>(ws), grid, form, any_zero, s);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return XENG_EHIP;
  }
  return XENG_OK;
}

int xeng_destroy(xeng_plan_t p) {
  if (!p) return XENG_OK;
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  for (int r = 0; r < kStageRing; ++r)
    if (p->copy_done[r]) (void)hipEventDestroy(p->copy_done[r]);
  if (p->d_insts) (void)hipFree(p->d_insts);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->h_insts) (void)hipHostFree(p->h_insts);
  if (p->gate_done) (void)hipEventDestroy(p->gate_done);
  if (p->d_gate_off) (void)hipFree(p->d_gate_off);
  if (p->d_runs) (void)hipFree(p->d_runs);
  if (p->h_gate_off) (void)hipHostFree(p->h_gate_off);
  if (p->h_runs) (void)hipHostFree(p->h_runs);
  if (p->d_vgate) (void)hipFree(p->d_vgate);
  if (p->h_vgate) (void)hipHostFree(p->h_vgate);
  if (p->d_seg_delay) (void)hipFree(p->d_seg_delay);
  if (p->d_blk_delay) (void)hipFree(p->d_blk_delay);
  if (p->d_shifted) (void)hipFree(p->d_shifted);
  if (p->d_chan_ws) (void)hipFree(p->d_chan_ws);
  if (p->chan_ws_used) (void)hipEventDestroy(p->chan_ws_used);
  if (p->d_fU) (void)hipFree(p->d_fU);
  if (p->d_fX) (void)hipFree(p->d_fX);
  if (p->d_fint) (void)hipFree(p->d_fint);
  if (p->d_fruns) (void)hipFree(p->d_fruns);
  if (p->d_wop) (void)hipFree(p->d_wop);
  if (p->d_bcorr) (void)hipFree(p->d_bcorr);
  if (p->tables_used) (void)hipEventDestroy(p->tables_used);
  delete p;
  return XENG_OK;
}

}  // extern "C"
