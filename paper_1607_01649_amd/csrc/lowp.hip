// Low-precision operands of the products with A (the precision growth of the
// sketch and projection GEMMs).
//
// A is converted once per factorisation (round to nearest even) into two
// copies: A16 (m x n, row-major) for A * X and A16T (n x m, row-major) for
// A^T * X, so both orientations read their operand with the contraction index
// contiguous; the transposed copy is written through a 64 x 64 LDS tile.  The
// same pass flags non-finite entries of A.
//
// The products themselves are in lpgemm.hip.
#include "internal.hpp"
#include "lowp_common.hpp"

namespace rsvd {

// ------------------------------------------------------------------ conversion

template <bool VEC>
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
    if (i < m) *reinterpret_cast<uint2*>(A16 + i * ld16 + j) = make_uint2(pack2(b[0], b[1]), pack2(b[2], b[3]));
  }
  if (nonfinite) atomicOr(flag, 1);
  __syncthreads();
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
    hipLaunchKernelGGL(to_bf16_kernel<true>, grid, dim3(256), 0, s, A, lda, m, n, A16, ld16, A16T, ldT, flag);
  else
    hipLaunchKernelGGL(to_bf16_kernel<false>, grid, dim3(256), 0, s, A, lda, m, n, A16, ld16, A16T, ldT, flag);
  return hipGetLastError();
}

}  // namespace rsvd
