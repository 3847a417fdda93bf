// Device building blocks of the X-engine kernels (gfx950 / CDNA4).
//
// The correlation of one channel is the complex Gram matrix V = X X^H of the
// N x T sample matrix X (Sec. I; Sec. IV-C, "Full Correlation").  Writing
// x = r + i m, the real and imaginary parts are two real contractions over the
// same operand rows (Sec. II, Eq. (1) counts one complex MAC per baseline and
// sample, i.e. four real MACs):
//
//     Re V_ij = sum_t r_i r_j + m_i m_j       = sum_k A_i[k] A_j[k]
//     Im V_ij = sum_t m_i r_j - r_i m_j       = sum_k A_i[k] Y_j[k]
//
// where a row A_n packs, for every block of 8 samples, the 8 real parts then
// the 8 imaginary parts, and Y_n is the same row with each block rotated to
// (-m, r).  Both are fed to the matrix cores (MFMA) as int8 (values -8..7) or
// as FP8 e4m3 codes (exact for those values).
//
// Operand staging.  Global memory holds samples[t][f][n] (n fastest), while an
// MFMA lane needs consecutive samples of one input.  Each workgroup therefore
// loads a chunk of KC = 64 samples x 128 inputs with 8-byte loads, transposes
// 8x8 byte blocks in registers (v_perm), splits the nibbles, removes the +8
// offset and stores 16-byte segments [r(8 samples), m(8 samples)] into LDS.
// A row of LDS holds the 8 segments of one input, padded to 144 bytes: eight
// lanes reading eight consecutive rows at one segment then hit disjoint banks,
// and the staging lanes, which write the 8 segments of a row side by side,
// too.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int BT = 128;        // tile edge (inputs)
constexpr int KC = 64;         // samples per staged chunk
constexpr int ROWB = 2 * KC + 16;  // bytes per LDS row (r and m of KC samples, padded)
constexpr int NTHREADS = 256;  // 4 waves: 2 x 2 wave tiles of 64 x 64
constexpr int BLOCK_LDS = BT * ROWB;          // one operand block, bytes
constexpr int STAGE_LDS = 2 * BLOCK_LDS;      // I block + J block
constexpr int LDS_BYTES = 2 * STAGE_LDS;      // double buffered

enum Form { FORM_I8 = 0, FORM_F8 = 1 };

// Byte offset of 16-byte segment q (0..7) of LDS row r.
__device__ __forceinline__ int seg_off(int r, int q) { return r * ROWB + 16 * q; }

// Transpose a 4x4 byte block: d[k] holds bytes (n0..n3) of time k; on return
// d[n] holds bytes (t0..t3) of input n.
__device__ __forceinline__ void transpose4x4(uint32_t& d0, uint32_t& d1, uint32_t& d2,
                                             uint32_t& d3) {
  const uint32_t s0 = __builtin_amdgcn_perm(d1, d0, 0x05010400u);
  const uint32_t s1 = __builtin_amdgcn_perm(d1, d0, 0x07030602u);
  const uint32_t s2 = __builtin_amdgcn_perm(d3, d2, 0x05010400u);
  const uint32_t s3 = __builtin_amdgcn_perm(d3, d2, 0x07030602u);
  d0 = __builtin_amdgcn_perm(s2, s0, 0x05040100u);
  d1 = __builtin_amdgcn_perm(s2, s0, 0x07060302u);
  d2 = __builtin_amdgcn_perm(s3, s1, 0x05040100u);
  d3 = __builtin_amdgcn_perm(s3, s1, 0x07060302u);
}

// Offset-binary nibbles (u = value + 8, four per word) to signed int8 bytes:
// per byte (u + 0x78) ^ 0x80 = u - 8 (mod 256); no carry crosses a byte.
__device__ __forceinline__ uint32_t nib_to_i8(uint32_t u) {
  return (u + 0x78787878u) ^ 0x80808080u;
}

// Offset-binary nibbles to FP8 e4m3 (OCP, bias 7) codes of u - 8.  Two 8-entry
// byte lookups (v_perm) for u < 8 and u >= 8, merged with a byte mask.
__device__ __forceinline__ uint32_t nib_to_f8(uint32_t u) {
  // codes of -8..-1 (u = 0..7) and of 0..7 (u = 8..15)
  const uint32_t neg_lo = 0xCACCCED0u, neg_hi = 0xB8C0C4C8u;
  const uint32_t pos_lo = 0x44403800u, pos_hi = 0x4E4C4A48u;
  const uint32_t sel = u & 0x07070707u;
  const uint32_t lo = __builtin_amdgcn_perm(neg_hi, neg_lo, sel);
  const uint32_t hi = __builtin_amdgcn_perm(pos_hi, pos_lo, sel);
  const uint32_t b3 = u & 0x08080808u;
  const uint32_t mask = (b3 << 5) - (b3 >> 3);  // 0xFF in bytes with u >= 8
  return (hi & mask) | (lo & ~mask);
}

// Negate four int8 bytes in [-8, 7]: ((~x ^ 0x80) + 1) ^ 0x80, carry-free.
__device__ __forceinline__ uint32_t neg_i8(uint32_t x) {
  return ((x ^ 0x7F7F7F7Fu) + 0x01010101u) ^ 0x80808080u;
}

}  // namespace xeng
