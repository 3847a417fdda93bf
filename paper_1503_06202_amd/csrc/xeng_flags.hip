// Flagged data (Sec. IV-A, "Data Flow"): lost packets and F-engine flags mark
// samples as invalid, and the count of such data renormalises the integrated
// matrices.  The kernels here run around the unchanged correlation:
//
//   scan     one workgroup per (channel, block of 64 time rows), lanes over
//            the flag words of a row: sets
//            every flagged sample to zero (code 0x88) in place, so that the
//            correlation adds nothing for it; counts rows with exactly one
//            invalid input per input; and turns rows with two or more invalid
//            inputs into rows of an event frame U whose correlation X adds
//            1 to X_ij for every such row where i and j are both invalid.
//            Identical rows of a block form one group: a group of m rows with
//            invalid set u adds m u u^T, written as one or two event rows
//            (a + ib) u with a^2 + b^2 summing to m (every m <= 64 is a sum of
//            four squares of at most 8, and -8 is a sample value); groups of
//            one row go two to an event row, one in the real part, one in the
//            imaginary part.  Saturated inputs and lost packets repeat the
//            same set over many rows, so U is usually a few rows per block.
//   pad      fills the unused tail of every channel's event rows with zeros
//            and writes the run table of the event correlation on the device.
//   (the 128 x 128 int8 MFMA kernel then correlates U into X)
//   counts   n_i = single-row count + X_ii is the number of invalid samples of
//            input i, and C_ij = T - n_i - n_j + X_ij the number of times both
//            are valid (C_ii = T - n_i).
//   normalize  V * scale / C in float64, rounded once to float32.
//
// Nothing here needs the host to know how many rows were flagged.  U has at
// most one row per time row (two thirds in the worst grouping); a frame
// without flags costs one read of the flag words.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xeng_internal.hpp"

namespace xeng {
namespace {

constexpr int kRows = 64;                 // time rows per workgroup of the scan
constexpr int kRowsPerWave = kRows / 4;   // its four waves take 16 rows each,
constexpr int kBatch = 4;                 // with the loads of 4 rows in flight
constexpr unsigned kZero4 = 0x88888888u;  // four samples of value 0 + 0i

// Bits 0..3 of x to bit 0 of bytes 0..3.
__device__ __forceinline__ unsigned spread4(unsigned x) {
  return (x & 1u) | ((x & 2u) << 7) | ((x & 4u) << 14) | ((x & 8u) << 21);
}

// Valid input bits of flag word w (inputs >= N mean nothing).
__device__ __forceinline__ unsigned word_mask(int w, int W, int N) {
  return (w == W - 1 && (N & 31)) ? ((1u << (N & 31)) - 1u) : 0xFFFFFFFFu;
}

// Flag bits of inputs i0 .. i0 + 15 (i0 a multiple of 16) of one row, with
// the bits of inputs >= N cleared.
__device__ __forceinline__ unsigned bits16(const uint32_t* frow, int i0, int N) {
  unsigned b = (frow[i0 >> 5] >> (i0 & 31)) & 0xFFFFu;
  if (N - i0 < 16) b &= (1u << (N - i0)) - 1u;
  return b;
}

// One 16-input piece of an event row: input k holds value va in its real part
// where bit k of `ba` is set, value vb in its imaginary part where bit k of
// `bb` is set, and 0 elsewhere.  Values 0..8 (8 is stored as -8).
__device__ __forceinline__ void store_piece(uint8_t* u, unsigned ba, unsigned bb, unsigned va,
                                            unsigned vb, int nvalid, bool vec) {
  const unsigned hi = (((va + 8) & 15u) << 4) * 0x01010101u;
  const unsigned lo = ((vb + 8) & 15u) * 0x01010101u;
  unsigned w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const unsigned sa = spread4(ba >> (4 * j)) * 0xF0u;  // high nibbles of the set bytes
    const unsigned sb = spread4(bb >> (4 * j)) * 0x0Fu;  // low nibbles
    w[j] = (kZero4 & ~(sa | sb)) | (hi & sa) | (lo & sb);
  }
  if (vec && nvalid == 16) {
    *reinterpret_cast<uint4*>(u) = make_uint4(w[0], w[1], w[2], w[3]);
  } else {
    for (int b = 0; b < nvalid; ++b) u[b] = (uint8_t)(w[b >> 2] >> (8 * (b & 3)));
  }
}

// m = a^2 + b^2 (+ c^2 + d^2), 0 <= a, b, c, d <= 8, in one row or two.
struct Weights {
  int8_t a, b, c, d, rows;
};
struct WeightTable {
  Weights w[65];
  constexpr WeightTable() : w{} {
    for (int m = 0; m <= 64; ++m) {
      w[m] = Weights{0, 0, 0, 0, 0};
      bool done = false;
      for (int a = 0; a <= 8 && !done; ++a)
        for (int b = 0; b <= a && !done; ++b)
          if (a * a + b * b == m) {
            w[m] = Weights{(int8_t)a, (int8_t)b, 0, 0, 1};
            done = true;
          }
      for (int a = 8; a >= 0 && !done; --a)
        for (int b = a; b >= 0 && !done; --b)
          for (int c = 0; c <= 8 && !done; ++c)
            for (int d = 0; d <= c && !done; ++d)
              if (a * a + b * b + c * c + d * d == m) {
                w[m] = Weights{(int8_t)a, (int8_t)b, (int8_t)c, (int8_t)d, 2};
                done = true;
              }
    }
  }
};
__constant__ WeightTable kWeights = WeightTable();

// Order-free row hash: the sum over nonzero words of a 64-bit mix of (word
// index, bits) (the finaliser of splitmix64).
__device__ __forceinline__ unsigned long long mix(unsigned v, int w) {
  unsigned long long x = ((unsigned long long)(unsigned)w << 32) | v;
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__global__ void flag_clear_kernel(FlagArgs a) {
  const long long n = (long long)a.F * a.N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    a.single[e] = 0;
    if (e < a.F) a.cnt[e] = 0;
  }
}

// One workgroup per (channel, block of 64 time rows).  VEC: sample and U rows
// are 16-byte aligned (N % 16 == 0, samples 16-byte aligned).
template <bool VEC>
__global__ void __launch_bounds__(256) flag_scan_kernel(FlagArgs a) {
  __shared__ int s_k[kRows], s_first[kRows], s_lead[kRows], s_bad[kRows];
  __shared__ unsigned long long s_hash[kRows];
  __shared__ int4 s_out[kRows];  // event rows: {row a, row b, value a, value b}
  __shared__ int s_nout, s_base;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = (int)(blockIdx.x % a.F);
  const int tb = (int)(blockIdx.x / a.F);
  const int nrows = min(kRows, a.T - tb * kRows);
  const long long row0 = (long long)tb * kRows * a.F + f;  // (t, f) row of block row 0
  const uint32_t* __restrict__ flags = a.flags;
  uint8_t* __restrict__ samples = a.samples;
  const int W = a.W, N = a.N;
  if (tid < kRows) {
    s_k[tid] = 0;
    s_first[tid] = 0x7fffffff;
    s_hash[tid] = 0;
    s_bad[tid] = 0;
    s_lead[tid] = -1;
  }
  __syncthreads();

  // A. per row: invalid inputs, the first of them and the hash; flagged
  //    samples become zero (code 0x88) so that the correlation skips them.
  //    Wave q takes rows 16 q .. 16 q + 15, lanes the words of a row; the
  //    loads of kBatch rows are issued together.
#pragma unroll 1
  for (int h = 0; h < kRowsPerWave; h += kBatch) {
    const int rbase = wave * kRowsPerWave + h;
    int k[kBatch], first[kBatch];
    unsigned long long hash[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      k[j] = 0;
      first[j] = 0x7fffffff;
      hash[j] = 0;
    }
    for (int w0 = 0; w0 < W; w0 += 64) {
      const int w = w0 + lane;
      const unsigned wm = w < W ? word_mask(w, W, N) : 0u;
      unsigned v[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        v[j] = (wm && rbase + j < nrows)
                   ? flags[(row0 + (long long)(rbase + j) * a.F) * W + w] & wm
                   : 0u;
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        unsigned x = v[j];
        if (!x) continue;
        k[j] += __builtin_popcount(x);
        first[j] = min(first[j], w * 32 + __builtin_ctz(x));
        hash[j] += mix(x, w);
        uint8_t* srow = samples + (row0 + (long long)(rbase + j) * a.F) * N + w * 32;
        if (VEC && x == 0xFFFFFFFFu && w * 32 + 32 <= N) {
          const uint4 z = make_uint4(kZero4, kZero4, kZero4, kZero4);
          reinterpret_cast<uint4*>(srow)[0] = z;
          reinterpret_cast<uint4*>(srow)[1] = z;
        } else {
          do {
            srow[__builtin_ctz(x)] = 0x88;
            x &= x - 1;
          } while (x);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      if (k[j]) {  // few lanes of a row hold invalid inputs: LDS atomics beat a reduction
        atomicAdd(&s_k[rbase + j], k[j]);
        atomicMin(&s_first[rbase + j], first[j]);
        atomicAdd(&s_hash[rbase + j], hash[j]);
      }
    }
  }
  __syncthreads();

  // B. wave 0, one lane per row: single-input rows are counted per input;
  //    rows with several invalid inputs are grouped by hash
  if (wave == 0) {
    const int k = lane < nrows ? s_k[lane] : 0;
    const int first = s_first[lane];
    const unsigned long long hash = s_hash[lane];
    unsigned long long ones = __ballot(k == 1);
    while (ones) {
      const int lead = __builtin_ctzll(ones);
      const int i1 = __shfl(first, lead);
      const unsigned long long match = __ballot(k == 1 && first == i1);
      if (lane == lead) atomicAdd(&a.single[(long long)f * N + i1], __popcll(match));
      ones &= ~match;
    }
    unsigned long long rem = __ballot(k >= 2);
    while (rem) {
      const int lead = __builtin_ctzll(rem);
      const unsigned hlo = __shfl((unsigned)hash, lead), hhi = __shfl((unsigned)(hash >> 32), lead);
      const unsigned long long match =
          __ballot(((rem >> lane) & 1ull) && (unsigned)hash == hlo && (unsigned)(hash >> 32) == hhi);
      if ((match >> lane) & 1ull) s_lead[lane] = lead;
      rem &= ~match;
    }
  }
  __syncthreads();

  // C. exact check: a row whose words differ from its leader's leaves the
  //    group (loads of kBatch rows in flight)
#pragma unroll 1
  for (int h = 0; h < kRowsPerWave; h += kBatch) {
    const int rbase = wave * kRowsPerWave + h;
    int lead[kBatch];
    bool any = false;
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int r = rbase + j, l = r < nrows ? s_lead[r] : -1;
      lead[j] = (l >= 0 && l != r) ? l : -1;
      any |= lead[j] >= 0;
    }
    if (!any) continue;  // uniform
    unsigned differ = 0;
    for (int w0 = 0; w0 < W; w0 += 64) {
      const int w = w0 + lane;
      const unsigned wm = w < W ? word_mask(w, W, N) : 0u;
      unsigned x[kBatch], y[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const bool on = wm && lead[j] >= 0;
        x[j] = on ? flags[(row0 + (long long)(rbase + j) * a.F) * W + w] : 0u;
        y[j] = on ? flags[(row0 + (long long)lead[j] * a.F) * W + w] : 0u;
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        if ((x[j] ^ y[j]) & wm) differ |= 1u << j;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (__ballot((differ >> j) & 1u) && lane == 0) s_bad[rbase + j] = 1;
  }
  __syncthreads();

  // D. wave 0: the event rows.  A group of m >= 2 identical rows is one or
  //    two rows (a + ib) u with weights summing to m; single rows (groups of
  //    one, including rows that left a group) go two to a row.
  if (wave == 0) {
    const int l = s_lead[lane];
    const int lead = (l >= 0 && s_bad[lane]) ? lane : l;  // -1: not an event row
    int mult = 0;
    {
      unsigned long long leaders = __ballot(lead == lane);
      while (leaders) {
        const int L = __builtin_ctzll(leaders);
        leaders &= leaders - 1;
        const int m = __popcll(__ballot(lead == L));
        if (lane == L) mult = m;
      }
    }
    unsigned long long heavy = __ballot(mult >= 2);
    unsigned long long lone = __ballot(mult == 1);
    int n = 0;
    while (heavy) {
      const int L = __builtin_ctzll(heavy);
      heavy &= heavy - 1;
      const Weights wt = kWeights.w[__shfl(mult, L)];
      if (lane == 0) {
        s_out[n] = make_int4(L, L, wt.a, wt.b);
        if (wt.rows == 2) s_out[n + 1] = make_int4(L, L, wt.c, wt.d);
      }
      n += wt.rows;
    }
    while (lone) {
      const int ra = __builtin_ctzll(lone);
      lone &= lone - 1;
      int rb = -1;
      if (lone) {
        rb = __builtin_ctzll(lone);
        lone &= lone - 1;
      }
      if (lane == 0) s_out[n] = make_int4(ra, rb, 1, rb < 0 ? 0 : 1);
      ++n;
    }
    if (lane == 0) {
      s_nout = n;
      s_base = n ? atomicAdd(&a.cnt[f], n) : 0;
    }
  }
  __syncthreads();

  // E. write the event rows (never more than the block's rows with several
  //    invalid inputs, so base + n <= cap)
  const int nout = s_nout, base = s_base;
  const int P = (N + 15) / 16;
  const int nv_last = N - (P - 1) * 16;
  for (int o = wave; o < nout; o += 4) {
    const long long urow = (long long)base + o;
    if (urow >= a.cap) break;  // not reached
    const int4 e = s_out[o];
    const long long ra = row0 + (long long)e.x * a.F;
    const long long rb = row0 + (long long)(e.y < 0 ? e.x : e.y) * a.F;
    uint8_t* u = a.U + (urow * a.F + f) * N;
    for (int p = lane; p < P; p += 64) {
      const unsigned ba = bits16(flags + ra * W, p * 16, N);
      const unsigned bb = e.y < 0 ? 0u : bits16(flags + rb * W, p * 16, N);
      store_piece(u + p * 16, ba, bb, (unsigned)e.z, (unsigned)e.w, p == P - 1 ? nv_last : 16,
                  VEC);
    }
  }
}

// R = event rows in use (the largest channel count, at most cap); rows
// [cnt[f], R) of channel f become zeros; block 0 writes R and the run table
// of the event correlation: segment k covers rows [k seg, min((k + 1) seg, R)),
// one run, or none when it starts at or past R.
template <bool VEC>
__global__ void flag_pad_kernel(FlagArgs a, int nseg, int seg) {
  __shared__ int smax;
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  int m = 0;
  for (int f = threadIdx.x; f < a.F; f += blockDim.x) m = max(m, a.cnt[f]);
  atomicMax(&smax, m);
  __syncthreads();
  const int R = (int)min((long long)smax, a.cap);
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) *a.R = R;
    for (int k = threadIdx.x; k < nseg; k += blockDim.x) {
      const int t0 = k * seg;
      const bool any = t0 < R;
      a.fgate_off[2 * k] = k;
      a.fgate_off[2 * k + 1] = any ? k + 1 : k;
      a.fruns[k] = make_int2(t0, any ? min(t0 + seg, R) : t0);
    }
  }
  const int P = (a.N + 15) / 16;
  const long long total = (long long)R * a.F * P;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(e % P);
    const long long rf = e / P;
    const int f = (int)(rf % a.F);
    const long long r = rf / a.F;
    if (r < a.cnt[f]) continue;
    store_piece(a.U + (r * a.F + f) * a.N + p * 16, 0u, 0u, 0u, 0u, min(16, a.N - p * 16), VEC);
  }
}

__device__ __forceinline__ long long diag_index(int i, int N) {
  return (long long)i * N - (long long)i * (i - 1) / 2;
}

__global__ void flag_n_kernel(FlagArgs a) {
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  const bool events = *a.R > 0;
  const long long n = (long long)a.F * a.N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int f = (int)(e / a.N), i = (int)(e % a.N);
    int v = a.single[e];
    if (events) v += a.X[2 * ((long long)f * NB + diag_index(i, a.N))];
    a.n[e] = v;
  }
}

// One workgroup per (channel, row i): baselines (i, j), j >= i.
__global__ void __launch_bounds__(256) flag_combine_kernel(FlagArgs a, int accumulate) {
  const long long row = blockIdx.x;
  const int f = (int)(row / a.N), i = (int)(row % a.N);
  const long long NB = (long long)a.N * (a.N + 1) / 2;
  const long long b0 = (long long)f * NB + diag_index(i, a.N);
  const bool events = *a.R > 0;
  const int ni = a.n[row];
  const int* nf = a.n + (long long)f * a.N;
  for (int j = i + threadIdx.x; j < a.N; j += blockDim.x) {
    const long long b = b0 + (j - i);
    int c = a.T - ni;
    if (j != i) c += (events ? a.X[2 * b] : 0) - nf[j];
    if (accumulate)
      a.counts[b] += c;
    else
      a.counts[b] = c;
  }
}

__global__ void normalize_kernel(const int2* __restrict__ vis, const int32_t* __restrict__ counts,
                                 long long n, double scale, float2* __restrict__ out) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = counts[e];
    float2 o = make_float2(0.f, 0.f);
    if (c > 0) {
      const int2 v = vis[e];
      const double dc = (double)c;
      o.x = (float)((double)v.x * scale / dc);
      o.y = (float)((double)v.y * scale / dc);
    }
    out[e] = o;
  }
}

int grid_for(long long n, int block, int cap = 4096) {
  const long long g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_flag_scan(const FlagArgs& a, int nseg, int seg, hipStream_t stream) {
  const long long nfn = (long long)a.F * a.N;
  hipLaunchKernelGGL(flag_clear_kernel, dim3(grid_for(nfn, 256)), dim3(256), 0, stream, a);
  const long long blocks = (long long)a.F * ((a.T + kRows - 1) / kRows);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool vec_u = (a.N % 16 == 0);
  const bool vec = vec_u && ((reinterpret_cast<uintptr_t>(a.samples) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL(flag_scan_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(flag_scan_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  if (vec_u)
    hipLaunchKernelGGL(flag_pad_kernel<true>, dim3(1024), dim3(256), 0, stream, a, nseg, seg);
  else
    hipLaunchKernelGGL(flag_pad_kernel<false>, dim3(1024), dim3(256), 0, stream, a, nseg, seg);
  return hipGetLastError();
}

hipError_t launch_flag_counts(const FlagArgs& a, int accumulate, hipStream_t stream) {
  const long long nfn = (long long)a.F * a.N;
  hipLaunchKernelGGL(flag_n_kernel, dim3(grid_for(nfn, 256)), dim3(256), 0, stream, a);
  if (nfn > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(flag_combine_kernel, dim3((unsigned)nfn), dim3(256), 0, stream, a,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_normalize(const int32_t* vis, const int32_t* counts, long long n, double scale,
                            float* out, hipStream_t stream) {
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, stream,
                     reinterpret_cast<const int2*>(vis), counts, n, scale,
                     reinterpret_cast<float2*>(out));
  return hipGetLastError();
}

}  // namespace xeng
