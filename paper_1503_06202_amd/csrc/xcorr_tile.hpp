// Device building blocks of the X-engine kernels (gfx950 / CDNA4).
//
// The correlation of one channel is the complex Gram matrix V = X X^H of the
// N x T sample matrix X (Sec. I; Sec. IV-C, "Full Correlation").  Writing
// x = r + i m, the real and imaginary parts are two real contractions over the
// same operand rows (Eq. (1) counts one complex MAC per baseline and sample,
// i.e. four real MACs):
//
//     Re V_ij = sum_t r_i r_j + m_i m_j       = sum_k A_i[k] A_j[k]
//     Im V_ij = sum_t m_i r_j - r_i m_j       = sum_k A_i[k] Y_j[k]
//
// where a row A_n packs, for every group of 8 samples, the 8 real parts then
// the 8 imaginary parts (or the reverse), and Y_n is the same row with each
// group rotated and one half negated.  Both are fed to the matrix cores
// (MFMA) as int8 or as FP8 e4m3 bytes.
//
// The 128 x 128 kernels feed the offset-binary codes u = v + 8 themselves (int8
// 0..15, or FP8 bytes that read u * 2^-9 and an operand scale of 2^9) and
// remove the offsets at the write from per-input sums of the codes; the
// 128 x 256 kernel converts the codes to the values -8..7 while staging
// (nib_to_i8, nib_to_f8 below).
//
// Operand staging.  Global memory holds samples[t][f][n] (n fastest).  A
// workgroup stages a chunk of KC = 64 samples of two blocks of 128 inputs:
// every thread loads 16-byte row pieces (sixteen inputs at one time; eight
// lanes cover a 128-byte row, so every load instruction reads whole cache
// lines) and stores them unchanged into an LDS plane laid out [t][n] as
// loaded, one byte per sample, with no transposition.  An MFMA lane needs
// eight consecutive samples of one input; the LDS transpose read
// (ds_read_b64_tr_b8) delivers exactly that: within a group of 16 lanes, lane
// i receives byte i & 7 of the 8 bytes addressed by lanes 2k + (i >> 3),
// k = 0..7, so lanes addressing rows t0..t0+7 at inputs n0..n0+15 receive,
// lane by lane, inputs n0+i at times t0..t0+7.  The lane then splits the
// nibbles of its 8 bytes into 8 real and 8 imaginary codes in registers, so
// that staging writes and transpose reads move one byte per sample, not two.
// Plane rows are 160 bytes (40 banks of 4 bytes): the 32 lanes of a transpose
// read pass (two 16-lane groups, 8 rows x 16 bytes each, 16 bytes apart) then
// cover all 64 banks once, and so do the 16 lanes of a staging write pass
// (two 128-byte rows 4 apart).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int BT = 128;                   // tile edge (inputs)
constexpr int KC = 64;                    // samples per staged chunk
constexpr int PROW = BT + 32;             // bytes per plane row (one time, 128 inputs, padded)
constexpr int PLANE = KC * PROW;          // one plane: the sample bytes of a block
constexpr int NTHREADS = 256;             // 4 waves: 2 x 2 wave tiles of 64 x 64
constexpr int BLOCK_LDS = PLANE;          // one operand block
constexpr int STAGE_LDS = 2 * BLOCK_LDS;  // I block + J block
constexpr int LDS_BYTES = 2 * STAGE_LDS;  // double buffered

enum Form { FORM_I8 = 0, FORM_F8 = 1 };

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

// Map a linear workgroup id b of G to a logical id so that consecutive
// logical ids, which share input rows, run on the same XCD: the dispatcher
// deals workgroups to the 8 XCDs round robin.
__device__ __forceinline__ int xcd_logical_id(int b, int G) {
  const int xcd = b & 7, slot = b >> 3, q = G >> 3, r = G & 7;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

// The real (high nibble) and imaginary (low nibble) codes of eight sample
// bytes, one code per byte.
__device__ __forceinline__ v2i hi_codes(v2i w) {
  return v2i{(int)(((uint32_t)w.x >> 4) & 0x0F0F0F0Fu), (int)(((uint32_t)w.y >> 4) & 0x0F0F0F0Fu)};
}
__device__ __forceinline__ v2i lo_codes(v2i w) {
  return v2i{(int)((uint32_t)w.x & 0x0F0F0F0Fu), (int)((uint32_t)w.y & 0x0F0F0F0Fu)};
}

// LDS transpose read of 8 bytes (see above); p must be 8-byte aligned.
__device__ __forceinline__ v2i lds_tr8(const uint8_t* p) {
  typedef v2i __attribute__((address_space(3))) * lds_v2i;
  return __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i)(p));
}

}  // namespace xeng
