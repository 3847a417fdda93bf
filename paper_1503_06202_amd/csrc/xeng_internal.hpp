// Internal interface between the C ABI (xeng_api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

// How a finished tile reaches vis: plain store, read-add-store (the
// workgroup owns the tile), or int32 atomic add (several workgroups share it).
// The persistent batch kernel turns WM_ATOMIC into WM_ATOMIC64 where vis is
// 8-byte aligned: one exact 64-bit atomic add per baseline instead of two
// 32-bit ones (see put_pairs in xcorr_device.hpp).
enum WriteMode { WM_STORE = 0, WM_ADD = 1, WM_ATOMIC = 2, WM_ATOMIC64 = 3 };

// Arguments of the tile kernel: one frame, all channels.
struct TileArgs {
  const uint8_t* samples;  // device [T][F][N]
  int32_t* vis;            // device [F][N(N+1)/2][2]
  int N, F;
  int t0, t1;          // integrated time range [t0, t1) of this launch
  int nt;              // tiles per edge, ceil(N / 128)
  int tiles_per_chan;  // nt (nt + 1) / 2
  int nslices;         // time slices per head tile
  int slice_len;       // samples per slice, a multiple of 64
  int write_mode;      // WM_STORE, WM_ADD or WM_ATOMIC: head items
  long long row_stride;  // F * N: bytes between consecutive time rows
  // Tiles are numbered g = f * tiles_per_chan + p.  Head tiles [0, head_tiles)
  // run as nslices slices each; the remaining (tail) tiles as tail_slices
  // slices of tail_len samples each, adding with int32 atomics (tail_mode).
  // Without a tail, head_tiles = F * tiles_per_chan and tail_slices = 0.
  int head_tiles;
  int tail_slices;
  int tail_len;
  int tail_mode;
  // time shifting: delays per 16-input segment and their maximum per
  // 128-input block (device), or NULL
  const int* seg_delay;
  const int* blk_delay;
  // 1: diagonal tiles split the sub-tile above the diagonal between two
  // waves and skip the block below it; 0: they keep the off-diagonal wave
  // roles (fast loads without time shifting only; others always split)
  int split_diag;
};

hipError_t launch_tiles(const TileArgs& a, int form, bool aligned, hipStream_t stream);

// Output gating: every (channel, tile, work gate g) integrates the runs
// runs[gate_off[g] .. gate_off[g + 1]) (absolute [begin, end) sample ranges)
// into the buffer vis + og * F * N(N+1) (gate-major output [G][F][N(N+1)/2][2]).
// Without vgate, work gate g is output gate og = g, written in write_mode.
// With vgate, vgate[g] = (og, mode): a gate whose runs, each integrated in
// whole chunks, hold more samples than one exact integration may is split
// into several work gates that add into its buffer with int32 atomics.
struct GatedArgs {
  const uint8_t* samples;
  int32_t* vis;
  int N, F, G;            // G: work gates of this launch
  int nt, tiles_per_chan;
  int write_mode;         // WM_STORE or WM_ADD (one work item per output tile)
  const int* gate_off;    // device [G + 1]
  const int2* runs;       // device [gate_off[G]]
  const int2* vgate;      // device [G] (output gate, write mode), or NULL
  long long row_stride;
  const int* seg_delay;   // time shifting, as in TileArgs
  const int* blk_delay;
  int skip_empty;         // 1: a gate without runs leaves its output untouched
};

hipError_t launch_gated(const GatedArgs& a, int form, bool aligned, hipStream_t stream);
// Clear the visibilities of tiles [first, first + count) (numbered as in
// TileArgs) before their slices add into them.
hipError_t launch_zero_tiles(int32_t* vis, int N, int tiles_per_chan, int nt, int first, int count,
                             hipStream_t stream);
// 128 x 256 tiles, one workgroup per CU; needs N % 16 == 0 and 16-byte rows.
// a.nt = ceil(N / 128), a.tiles_per_chan = wide tiles per channel.
hipError_t launch_wide(const TileArgs& a, int form, hipStream_t stream);
hipError_t launch_zero(int32_t* p, long long n, hipStream_t stream);

// Flagged data: the scan, pad and count kernels around the correlation.
struct FlagArgs {
  uint8_t* samples;        // device [T][F][N]; flagged samples are set to 0x88
  const uint32_t* flags;   // device [T][F][W]; bit i % 32 of word i / 32 = invalid
  int N, F, T, W;          // W = ceil(N / 32)
  uint8_t* U;              // device [cap][F][N]: event rows, two flagged rows each
  long long cap;           // event rows available per channel
  int* cnt;                // device [F]: event rows used per channel
  int* single;             // device [F][N]: rows whose only invalid input is i
  int* n;                  // device [F][N]: invalid samples per input
  int* R;                  // device [1]: event rows correlated (max of cnt, <= cap)
  int32_t* X;              // device [F][N(N+1)/2][2]: correlation of U
  int* fgate_off;          // device [2 nseg]: run table of the event correlation
  int2* fruns;             // device [nseg]
  int32_t* counts;         // device [F][N(N+1)/2]: valid pairs per baseline
};

// Clear the per-call counters, scan the flags (zeroing flagged samples and
// building U), then pad U and write R and the run table (nseg segments of seg
// rows).
hipError_t launch_flag_scan(const FlagArgs& a, int nseg, int seg, hipStream_t stream);
// After the correlation of U into X: invalid counts per input, then counts.
hipError_t launch_flag_counts(const FlagArgs& a, int accumulate, hipStream_t stream);
// out[e] = vis[e] * scale / counts[e] (float64, rounded to float32), 0 where
// counts[e] == 0; n baselines.
hipError_t launch_normalize(const int32_t* vis, const int32_t* counts, long long n, double scale,
                            float* out, hipStream_t stream);

// Time shifting by a copy: dst[t][f][16 g + e] = src[t - seg_delay[g]][f][16 g + e]
// for t < T; rows before src are its history.
hipError_t launch_shift_copy(const uint8_t* src, uint8_t* dst, int N, int F, int T,
                             const int* seg_delay, hipStream_t stream);

// Discrete beamforming: one launch covers the component tiles c0 .. c0 + nb - 1
// (32 columns of the real contraction each; column 2b + comp is beam b's real
// (comp 0) or imaginary (comp 1) part) over T rows starting at `samples`.
struct BeamArgs {
  const uint8_t* samples;  // device, this launch's first row of [T][F][N]
  int32_t* beams;          // device, the same row of [T][F][B][2]
  const void* wop;         // device weight operands [F][S][8][NBT][64 lanes][16 bytes]
  const int* corr;         // device [F][NBT * 32]: 8 times the column sums of the operands
  int N, F, T, B;
  int S;                   // steps of 128 inputs: ceil(N / 128)
  int NBT;                 // component tiles in all: ceil(2B / 32)
  int c0;                  // first component tile of this launch
  int tblocks;             // set by launch_beams
};

// Rows of one workgroup for nb component tiles per launch (at most 256).
int beam_rows_per_block(int nb, bool aligned);
// nb = 1..4 component tiles; aligned: N % 16 == 0 and samples 16-byte
// aligned.  The host keeps (T + rows per workgroup) F N below 2^31.
hipError_t launch_beams(BeamArgs a, int nb, bool aligned, hipStream_t stream);

// One work item of the batched persistent kernel.
struct BatchItem {
  int inst;   // instance index
  int f;      // channel
  int I, J;   // tile
  int t0, t1; // time range
  int mode;   // write mode
  int pad;
};

// Per-instance descriptor on the device.
struct BatchInst {
  const uint8_t* samples;  // device [T][F][N]
  int32_t* vis;            // device [F][N(N+1)/2][2]
  int N, F, T;
  int aligned;  // N % 16 == 0, samples 16-byte aligned, F * N <= 2^26
  int zero;     // clear vis before the launch (its tiles are integrated by atomic adds)
  int pad;
};

// Clear the outputs flagged `zero` and reset the work counter, then run the
// persistent kernel with `grid` workgroups over the item list.
hipError_t launch_batch(const BatchInst* insts, int ninst, const BatchItem* items, int nitems,
                        int* counter, int grid, int form, bool any_zero, hipStream_t stream);

}  // namespace xeng
