// Block-scaled FP8 (OCP E4M3) operands of the products with A.
//
// Format: E4M3 with bias 7, 3 mantissa bits, largest finite value 448, no
// infinities (0x7F / 0xFF are NaN); round to nearest, ties to even,
// saturating at +-448.  Block scales are powers of two: a block with largest
// magnitude amax stores round(x / 2^e) with e the least integer such that
// amax <= 448 2^e (e = 0 for an all-zero block).
//
// A (FP32, m x n) is converted once per factorisation into A8 (m x ld8) and
// its transpose A8T (n x ldT) with one scale per 128 x 128 tile, shared by
// both copies, so A X and A^T X read the same quantised values with the
// contraction index contiguous.  The thin FP32 operand X of a product is
// quantised as it is staged: one scale per 128-row segment of each column.
//
// The product itself is in lpgemm.hip.
#include <algorithm>

#include "internal.hpp"
#include "lowp_common.hpp"

namespace rsvd {


// ------------------------------------------------------------------ conversion

// One 128 x 128 tile per block (256 threads): scale, A8 rows, and A8T rows through LDS.
template <bool VEC, bool TILED>
__global__ __launch_bounds__(256) void to_fp8_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                     uint8_t* __restrict__ A8, int64_t ld8, uint8_t* __restrict__ A8T,
                                                     int64_t ldT, float* __restrict__ scale, int ntc,
                                                     int* __restrict__ flag) {
  __shared__ __align__(16) uint8_t tile[128][132];
  __shared__ float wmax[4];
  const int t = threadIdx.x;
  const int c4 = t & 31, rg = t >> 5;
  const int64_t i0 = (int64_t)blockIdx.y * 128, j0 = (int64_t)blockIdx.x * 128;
  float v[16][4];
  float mx = 0.f;
  bool nonfinite = false;
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int64_t i = i0 + rg + 8 * rr, j = j0 + 4 * c4;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[rr][e] = 0.f;
    if (i < m) {
      const float* p = A + i * lda + j;
      if (VEC && j + 4 <= n) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[rr][0] = q.x; v[rr][1] = q.y; v[rr][2] = q.z; v[rr][3] = q.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[rr][e] = (j + e < n) ? p[e] : 0.f;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      nonfinite |= !isfinite(v[rr][e]);
      mx = fmaxf(mx, fabsf(v[rr][e]));
    }
  }
  if (nonfinite) atomicOr(flag, 1);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((t & 63) == 0) wmax[t >> 6] = mx;
  __syncthreads();
  const float amax = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
  const int ex = fp8_scale_exp(amax);
  // (the tiled form's grid reaches past the scale table to zero the padding of the last row block)
  if (t == 0 && (!TILED || (i0 < ldT && j0 < ld8))) scale[(int64_t)blockIdx.y * ntc + blockIdx.x] = ldexpf(1.0f, ex);
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int ii = rg + 8 * rr;
    const int64_t i = i0 + ii;
    const uint32_t w = f32x4_to_e4m3(ldexpf(v[rr][0], -ex), ldexpf(v[rr][1], -ex), ldexpf(v[rr][2], -ex),
                                     ldexpf(v[rr][3], -ex));
    *reinterpret_cast<uint32_t*>(&tile[ii][4 * c4]) = w;   // row pitch 132: 4-byte aligned
    if (!TILED && i < m) *reinterpret_cast<uint32_t*>(A8 + i * ld8 + j0 + 4 * c4) = w;
  }
  __syncthreads();
  if constexpr (TILED) {
    // 16-byte units (16 codes): A8 (row i0 + ii, indices j0 + 16 cu ..) and A8T (row j0 + jj, indices i0 + 16 ru ..),
    // four of each per thread
    const int64_t rbA = lp_tiled_rows(m) / kTileRows, rbT = lp_tiled_rows(n) / kTileRows;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int u = t + 256 * h;
      const int ii = u >> 3, cu = u & 7;
      const int64_t r = i0 + ii, k = j0 + 16 * cu;
      if (r < rbA * kTileRows && k < ld8) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&tile[ii][16 * cu]);
        *reinterpret_cast<uint4*>(A8 + 16 * lp_tiled_unit<1>(r, k, rbA)) = make_uint4(src[0], src[1], src[2], src[3]);
      }
      const int jj = u >> 3, ru = u & 7;
      const int64_t rt = j0 + jj, kt = i0 + 16 * ru;
      if (rt < rbT * kTileRows && kt < ldT) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r0 = 16 * ru + 4 * q;
          w[q] = (uint32_t)tile[r0][jj] | ((uint32_t)tile[r0 + 1][jj] << 8) | ((uint32_t)tile[r0 + 2][jj] << 16) |
                 ((uint32_t)tile[r0 + 3][jj] << 24);
        }
        *reinterpret_cast<uint4*>(A8T + 16 * lp_tiled_unit<1>(rt, kt, rbT)) = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    return;
  }
  // transposed: thread t writes 64 bytes of row j0 + t/2 of A8T (columns i0 + 64 (t%2) ..)
  const int jj = t >> 1, half = t & 1;
  const int64_t j = j0 + jj;
  if (j < n) {
    uint32_t w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r0 = 64 * half + 4 * q;
      w[q] = (uint32_t)tile[r0][jj] | ((uint32_t)tile[r0 + 1][jj] << 8) | ((uint32_t)tile[r0 + 2][jj] << 16) |
             ((uint32_t)tile[r0 + 3][jj] << 24);
    }
    uint4* o = reinterpret_cast<uint4*>(A8T + j * ldT + i0 + 64 * half);
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  }
}

hipError_t launch_to_fp8(const float* A, int64_t lda, int64_t m, int64_t n, uint8_t* A8, int64_t ld8, uint8_t* A8T,
                         int64_t ldT, float* scale, int* flag, hipStream_t s) {
  if (ld8 % 128 != 0 || ldT % 128 != 0 || ld8 < n || ldT < m) return hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(A8) & 15) != 0 || (reinterpret_cast<uintptr_t>(A8T) & 15) != 0)
    return hipErrorInvalidValue;
  const int ntc = (int)(ld8 / 128);
  dim3 grid((unsigned)ntc, (unsigned)(ldT / 128));
  const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL((to_fp8_kernel<true, false>), grid, dim3(256), 0, s, A, lda, m, n, A8, ld8, A8T, ldT, scale, ntc,
                       flag);
  else
    hipLaunchKernelGGL((to_fp8_kernel<false, false>), grid, dim3(256), 0, s, A, lda, m, n, A8, ld8, A8T, ldT, scale,
                       ntc, flag);
  return hipGetLastError();
}

size_t fp8_tiled_bytes(int64_t rows, int64_t K) {
  return (size_t)lp_tiled_rows(rows) * (size_t)((K + kTileK - 1) / kTileK * kTileK);
}

// The same codes and scales with A8 and A8T in the tiled layout (lowp_common.hpp); the scale table is that of
// launch_to_fp8 ((ldT / 128) x (ld8 / 128), ld8 = n and ldT = m rounded up to 128).
hipError_t launch_to_fp8_tiled(const float* A, int64_t lda, int64_t m, int64_t n, uint8_t* A8, uint8_t* A8T,
                               float* scale, int* flag, hipStream_t s) {
  if ((reinterpret_cast<uintptr_t>(A8) & 15) != 0 || (reinterpret_cast<uintptr_t>(A8T) & 15) != 0)
    return hipErrorInvalidValue;
  const int64_t ld8 = (n + kTileK - 1) / kTileK * kTileK, ldT = (m + kTileK - 1) / kTileK * kTileK;
  const int ntc = (int)(ld8 / 128);
  const int64_t cols = std::max(ld8, lp_tiled_rows(n)), rows = std::max(ldT, lp_tiled_rows(m));
  dim3 grid((unsigned)(cols / 128), (unsigned)(rows / 128));
  const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL((to_fp8_kernel<true, true>), grid, dim3(256), 0, s, A, lda, m, n, A8, ld8, A8T, ldT, scale, ntc,
                       flag);
  else
    hipLaunchKernelGGL((to_fp8_kernel<false, true>), grid, dim3(256), 0, s, A, lda, m, n, A8, ld8, A8T, ldT, scale,
                       ntc, flag);
  return hipGetLastError();
}

}  // namespace rsvd
