// Low-precision operands of the products with A (the precision growth of the
// sketch and projection GEMMs).
//
// A is converted once per factorisation (round to nearest even) into two
// copies: A16 (m x n, row-major) for A * X and A16T (n x m, row-major) for
// A^T * X, so both orientations read their operand with the contraction index
// contiguous; the transposed copy is written through a 64 x 64 LDS tile.  The
// same pass flags non-finite entries of A.
//
// nn_bf16_kernel: out[split][c][r] = sum_{j in split} A16[r][j] X(j, c) on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  X is an FP32 panel,
// rounded to bf16 as it is staged in LDS.  Within each 128-wide K chunk a lane
// loads 64 contiguous bytes of its row (32 values) and feeds them to four
// MFMAs; the contraction index is permuted accordingly (k = 32 g + 8 t + e
// for lane group g, MFMA t, element e) on both operands.
#include "internal.hpp"

namespace rsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

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

// ------------------------------------------------------------------ product

constexpr int KCB = 128;   // K rows staged per iteration

template <int NB>
__global__ __launch_bounds__(256) void nn_bf16_kernel(const uint16_t* __restrict__ A, int64_t lda, int64_t rows,
                                                      int64_t K, const float* __restrict__ X, int64_t ldx, int ncols,
                                                      float* __restrict__ out, int64_t ldo, int64_t part_stride,
                                                      int64_t kchunk) {
  __shared__ u32x4 xs[NB * 4 * 64];   // (cb, t, lane) -> 8 bf16
  typedef Mma<float> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * 128 + wave * 32;
  const int split = blockIdx.y;
  const int cg0 = blockIdx.z * NB * 16;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);

  f32x4 acc[2][NB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = M::zero();

  for (int64_t k0 = kbeg; k0 < kend; k0 += KCB) {
    // stage X rows [k0, k0+128) x columns [cg0, cg0 + 16 NB) as bf16 fragments
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = threadIdx.x + 256 * u;
      const int cl = it >> 4, ch = it & 15;
      const int c = cg0 + cl;
      const int64_t kk = k0 + 8 * ch;
      float v[8];
      if (c < ncols && kk + 8 <= kend) {
        const float* p = X + (int64_t)c * ldx + kk;
        float4 q0 = *reinterpret_cast<const float4*>(p);
        float4 q1 = *reinterpret_cast<const float4*>(p + 4);
        v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w; v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (c < ncols && kk + e < kend) ? X[(int64_t)c * ldx + kk + e] : 0.f;
      }
      u32x4 w;
      w[0] = pack2(f32_to_bf16_rne(v[0]), f32_to_bf16_rne(v[1]));
      w[1] = pack2(f32_to_bf16_rne(v[2]), f32_to_bf16_rne(v[3]));
      w[2] = pack2(f32_to_bf16_rne(v[4]), f32_to_bf16_rne(v[5]));
      w[3] = pack2(f32_to_bf16_rne(v[6]), f32_to_bf16_rne(v[7]));
      const int cb = cl >> 4, cli = cl & 15, gg = ch >> 2, tt = ch & 3;
      xs[(cb * 4 + tt) * 64 + cli + 16 * gg] = w;
    }
    // A: this lane's 32 contiguous values of rows rbase + 16 rb + li
    u32x4 a[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t r = rbase + 16 * rb + li;
      if (r < rows) {
        const u32x4* p = reinterpret_cast<const u32x4*>(A + r * lda + k0 + 32 * g);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) a[rb][tt] = p[tt];
      } else {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) a[rb][tt] = u32x4{0u, 0u, 0u, 0u};
      }
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      bf16x8 b[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) b[cb] = __builtin_bit_cast(bf16x8, xs[(cb * 4 + tt) * 64 + lane]);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        bf16x8 av = __builtin_bit_cast(bf16x8, a[rb][tt]);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[cb], acc[rb][cb], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  float* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = cg0 + cb * 16 + li;
      if (c >= ncols) continue;
      const int64_t r = rbase + rb * 16 + 4 * g;
      float* p = o + (int64_t)c * ldo + r;
      if (r + 4 <= rows) {
        *reinterpret_cast<float4*>(p) = make_float4(acc[rb][cb][0], acc[rb][cb][1], acc[rb][cb][2], acc[rb][cb][3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (r + e < rows) p[e] = acc[rb][cb][e];
      }
    }
}

int lp_splits_used(int64_t K, int splits) {
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + KCB - 1) / KCB * KCB;
  if (kchunk < KCB) kchunk = KCB;
  int used = (int)((K + kchunk - 1) / kchunk);
  return used < 1 ? 1 : used;
}

hipError_t launch_nn_bf16(const uint16_t* A, int64_t lda, int64_t rows, int64_t K, const float* X, int64_t ldx,
                          int ncols, float* out, int64_t ldo, int64_t part_stride, int splits, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (lda % 128 != 0 || lda < K || (reinterpret_cast<uintptr_t>(A) & 15) != 0 || ldx % 4 != 0)
    return hipErrorInvalidValue;
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + KCB - 1) / KCB * KCB;
  if (kchunk < KCB) kchunk = KCB;
  int used = (int)((K + kchunk - 1) / kchunk);
  int nb = (ncols + 15) / 16;
  nb = nb > 8 ? 8 : nb;
  int groups = (ncols + nb * 16 - 1) / (nb * 16);
  dim3 grid((unsigned)((rows + 127) / 128), (unsigned)used, (unsigned)groups);
  switch (nb) {
#define RSVD_BF16_CASE(NBV) \
    case NBV: hipLaunchKernelGGL(nn_bf16_kernel<NBV>, grid, dim3(256), 0, s, A, lda, rows, K, X, ldx, ncols, out, \
                                 ldo, part_stride, kchunk); break;
    RSVD_BF16_CASE(1) RSVD_BF16_CASE(2) RSVD_BF16_CASE(3) RSVD_BF16_CASE(4)
    RSVD_BF16_CASE(5) RSVD_BF16_CASE(6) RSVD_BF16_CASE(7) default: RSVD_BF16_CASE(8)
#undef RSVD_BF16_CASE
  }
  return hipGetLastError();
}

}  // namespace rsvd
