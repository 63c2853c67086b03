// Device helpers of the low-precision operand formats (bfloat16 and OCP FP8
// E4M3 with power-of-two block scales), shared by the conversion and product
// kernels.
#pragma once

#include "device_common.hpp"

namespace rsvd {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// bfloat16 of x, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// E4M3 code of x, round to nearest even, saturating; NaN -> 0x7F (with sign).
__device__ __forceinline__ uint32_t f32_to_e4m3(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sgn = (u >> 24) & 0x80u;
  const uint32_t au = u & 0x7fffffffu;
  if (au > 0x7f800000u) return sgn | 0x7Fu;
  const float a = __uint_as_float(au);
  if (a >= 448.0f) return sgn | 0x7Eu;
  if (a < 0.015625f) return sgn | (uint32_t)rintf(a * 512.0f);   // multiples of 2^-9 (rint: ties to even)
  const uint32_t r = au + 0x7FFFFu + ((au >> 20) & 1u);           // keep 3 mantissa bits, ties to even
  const uint32_t e = ((r >> 23) & 0xFFu) - 127u + 7u;
  return sgn | (e << 3) | ((r >> 20) & 7u);
}

// Four E4M3 codes (x0 in the low byte), each the code f32_to_e4m3 gives: gfx950's packed conversion when all
// four are finite with magnitude at most 448 (round to nearest even with E4M3 subnormals: the same code as
// f32_to_e4m3 for every such value of either sign, checked on the device over all of them), the software
// rounding otherwise (non-finite and saturated values).  The scaled operands of the products always take the
// hardware path.
__device__ __forceinline__ uint32_t f32x4_to_e4m3(float x0, float x1, float x2, float x3) {
  if (fabsf(x0) <= 448.0f && fabsf(x1) <= 448.0f && fabsf(x2) <= 448.0f && fabsf(x3) <= 448.0f) {
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x0, x1, 0, false);
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x2, x3, lo, true);
  }
  return f32_to_e4m3(x0) | (f32_to_e4m3(x1) << 8) | (f32_to_e4m3(x2) << 16) | (f32_to_e4m3(x3) << 24);
}

// Least e with amax <= 448 2^e (0 for amax == 0): amax = f 2^E, f in [0.5, 1), 448 = 0.875 2^9.
// Exponents are kept in [-127, 127], the range of an E8M0 scale (the MFMA's block-scale operand); only blocks
// whose largest magnitude is below 448 2^-127 reach the lower limit.
__device__ __forceinline__ int fp8_scale_exp(float amax) {
  if (!(amax > 0.0f)) return 0;
  int E;
  const float f = frexpf(amax, &E);
  const int e = f <= 0.875f ? E - 9 : E - 8;
  return e < -127 ? -127 : e;
}

// Tiled layout of a low-precision copy (rows x K, elements of EB bytes) for the library's products: blocks of
// 256 rows x 128 contraction indices (one workgroup's rows and one chunk, 32 KB per byte of element width),
// block (c, rb) = (k / 128, r / 256) at block index c * rblocks + rb, so that a workgroup streams one
// contiguous block per chunk; inside a block, 16-byte units in the order the product's waves load them:
// wave w = (r % 256) / 64, row block b = (r % 64) / 16, unit a of the lane's 32 contraction indices, lane
// 16 g + (r % 16) with g = (k % 128) / 32.  Rows past the end and indices past K are zero.
constexpr int kTileRows = 256;
constexpr int kTileK = 128;
template <int EB>
__host__ __device__ __forceinline__ int64_t lp_tiled_unit(int64_t r, int64_t k, int64_t rblocks) {
  constexpr int EPU = 16 / EB;       // elements per 16-byte unit
  constexpr int AW = 32 / EPU;       // units per lane per row block per chunk
  constexpr int UPB = kTileRows * kTileK * EB / 16;
  const int64_t c = k / kTileK, rb = r / kTileRows;
  const int rr = (int)(r - rb * kTileRows), kk = (int)(k - c * kTileK);
  const int w = rr >> 6, b = (rr >> 4) & 3, li = rr & 15, g = kk >> 5, a = (kk & 31) / EPU;
  return (c * rblocks + rb) * UPB + ((w * 4 + b) * AW + a) * 64 + g * 16 + li;
}
__host__ __device__ __forceinline__ int64_t lp_tiled_rows(int64_t rows) {
  return (rows + kTileRows - 1) / kTileRows * kTileRows;
}

}  // namespace rsvd
