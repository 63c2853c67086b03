// Low-precision operands of the products with A (the precision growth of the
// sketch and projection GEMMs).
//
// A is converted once per factorisation (round to nearest even) into two
// copies: A16 (m x n) for A * X and A16T (n x m) for A^T * X, so both
// orientations read their operand with the contraction index contiguous; the
// transposed copy is written through a 64 x 64 LDS tile.  The same pass flags
// non-finite entries of A.  Two layouts: row-major (the kernel-level entry
// points), or the tiled layout of lowp_common.hpp that the library's products
// stream (each workgroup reads one contiguous 64 KB block per chunk instead of
// 256-byte pieces of 256 rows: 4.5 -> 5.5 TB/s for the product).
//
// The products themselves are in lpgemm.hip.
#include <algorithm>

#include "internal.hpp"
#include "lowp_common.hpp"

namespace rsvd {

// ------------------------------------------------------------------ conversion

template <bool VEC, bool TILED>
__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      uint16_t* __restrict__ A16, int64_t ld16,
                                                      uint16_t* __restrict__ A16T, int64_t ldT,
                                                      int* __restrict__ flag) {
  __shared__ uint16_t tile[64][66];
  const int t = threadIdx.x;
  const int c4 = t & 15, rg = t >> 4;
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  bool nonfinite = false;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int ii = rg * 4 + rr;
    const int64_t i = i0 + ii, j = j0 + 4 * c4;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < m) {
      const float* p = A + i * lda + j;
      if (VEC && j + 4 <= n) {
        float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (j + e < n) ? p[e] : 0.f;
      }
    }
    uint16_t b[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      nonfinite |= !isfinite(v[e]);
      b[e] = f32_to_bf16_rne(v[e]);
      tile[ii][4 * c4 + e] = b[e];
    }
    if (!TILED && i < m)
      *reinterpret_cast<uint2*>(A16 + i * ld16 + j) = make_uint2(pack2(b[0], b[1]), pack2(b[2], b[3]));
  }
  if (nonfinite) atomicOr(flag, 1);
  __syncthreads();
  if constexpr (TILED) {
    // 16-byte units: A16 (row i0 + ii, indices j0 + 8 cu ..) and A16T (row j0 + jj, indices i0 + 8 ru ..), two of
    // each per thread; rows up to the tiled row count, indices up to the padded width, zeros past m and n
    const int64_t rbA = lp_tiled_rows(m) / kTileRows, rbT = lp_tiled_rows(n) / kTileRows;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int u = t + 256 * h;
      const int ii = u >> 3, cu = u & 7;
      const int64_t r = i0 + ii, k = j0 + 8 * cu;
      if (r < rbA * kTileRows && k < ld16) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&tile[ii][8 * cu]);
        *reinterpret_cast<uint4*>(A16 + 8 * lp_tiled_unit<2>(r, k, rbA)) = make_uint4(src[0], src[1], src[2], src[3]);
      }
      const int jj = u >> 3, ru = u & 7;
      const int64_t rt = j0 + jj, kt = i0 + 8 * ru;
      if (rt < rbT * kTileRows && kt < ldT) {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = pack2(tile[8 * ru + 2 * e][jj], tile[8 * ru + 2 * e + 1][jj]);
        *reinterpret_cast<uint4*>(A16T + 8 * lp_tiled_unit<2>(rt, kt, rbT)) = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    return;
  }
  const int jj = t >> 2, ic = t & 3;
  const int64_t j = j0 + jj;
  if (j < n) {
    uint32_t w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = pack2(tile[16 * ic + 2 * e][jj], tile[16 * ic + 2 * e + 1][jj]);
    uint4* o = reinterpret_cast<uint4*>(A16T + j * ldT + i0 + 16 * ic);
    o[0] = make_uint4(w[0], w[1], w[2], w[3]);
    o[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
}

hipError_t launch_to_bf16(const float* A, int64_t lda, int64_t m, int64_t n, uint16_t* A16, int64_t ld16,
                          uint16_t* A16T, int64_t ldT, int* flag, hipStream_t s) {
  if (ld16 % 128 != 0 || ldT % 128 != 0 || ld16 < n || ldT < m) return hipErrorInvalidValue;
  dim3 grid((unsigned)(ld16 / 64), (unsigned)(ldT / 64));
  bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL((to_bf16_kernel<true, false>), grid, dim3(256), 0, s, A, lda, m, n, A16, ld16, A16T, ldT, flag);
  else
    hipLaunchKernelGGL((to_bf16_kernel<false, false>), grid, dim3(256), 0, s, A, lda, m, n, A16, ld16, A16T, ldT,
                       flag);
  return hipGetLastError();
}

size_t bf16_tiled_bytes(int64_t rows, int64_t K) {
  return (size_t)lp_tiled_rows(rows) * (size_t)((K + kTileK - 1) / kTileK * kTileK) * 2;
}

hipError_t launch_to_bf16_tiled(const float* A, int64_t lda, int64_t m, int64_t n, uint16_t* A16, uint16_t* A16T,
                                int* flag, hipStream_t s) {
  if ((reinterpret_cast<uintptr_t>(A16) & 15) != 0 || (reinterpret_cast<uintptr_t>(A16T) & 15) != 0)
    return hipErrorInvalidValue;
  const int64_t ld16 = (n + kTileK - 1) / kTileK * kTileK, ldT = (m + kTileK - 1) / kTileK * kTileK;
  const int64_t cols = std::max(ld16, lp_tiled_rows(n)), rows = std::max(ldT, lp_tiled_rows(m));
  dim3 grid((unsigned)(cols / 64), (unsigned)(rows / 64));
  bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL((to_bf16_kernel<true, true>), grid, dim3(256), 0, s, A, lda, m, n, A16, ld16, A16T, ldT, flag);
  else
    hipLaunchKernelGGL((to_bf16_kernel<false, true>), grid, dim3(256), 0, s, A, lda, m, n, A16, ld16, A16T, ldT, flag);
  return hipGetLastError();
}

}  // namespace rsvd
