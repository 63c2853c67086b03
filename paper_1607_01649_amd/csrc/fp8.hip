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
// nn_fp8_kernel: out[split][c][r] = sum_kb sA(r, kb) sX(kb, c) sum_{k in kb}
// A8[r][k] X8[k][c]: each 128-wide K block is one A tile column and one X
// segment, so its partial product comes from four v_mfma_f32_16x16x32_fp8_fp8
// (FP32 accumulation, OCP E4M3 operands on gfx950) into a fresh accumulator
// and is added with the product of the two scales.  Lane layout as in the
// bf16 kernel: lane group g feeds contraction indices 32 g + 8 t + e.
#include "internal.hpp"

namespace rsvd {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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

// Least e with amax <= 448 2^e (0 for amax == 0): amax = f 2^E, f in [0.5, 1), 448 = 0.875 2^9.
__device__ __forceinline__ int fp8_scale_exp(float amax) {
  if (!(amax > 0.0f)) return 0;
  int E;
  const float f = frexpf(amax, &E);
  return f <= 0.875f ? E - 9 : E - 8;
}

// ------------------------------------------------------------------ conversion

// One 128 x 128 tile per block (256 threads): scale, A8 rows, and A8T rows through LDS.
template <bool VEC>
__global__ __launch_bounds__(256) void to_fp8_kernel(const float* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                     uint8_t* __restrict__ A8, int64_t ld8, uint8_t* __restrict__ A8T,
                                                     int64_t ldT, float* __restrict__ scale, int ntc,
                                                     int* __restrict__ flag) {
  __shared__ uint8_t tile[128][132];
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
  if (t == 0) scale[(int64_t)blockIdx.y * ntc + blockIdx.x] = ldexpf(1.0f, ex);
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int ii = rg + 8 * rr;
    const int64_t i = i0 + ii;
    uint32_t w = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t c = f32_to_e4m3(ldexpf(v[rr][e], -ex));
      tile[ii][4 * c4 + e] = (uint8_t)c;
      w |= c << (8 * e);
    }
    if (i < m) *reinterpret_cast<uint32_t*>(A8 + i * ld8 + j0 + 4 * c4) = w;
  }
  __syncthreads();
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
    hipLaunchKernelGGL(to_fp8_kernel<true>, grid, dim3(256), 0, s, A, lda, m, n, A8, ld8, A8T, ldT, scale, ntc, flag);
  else
    hipLaunchKernelGGL(to_fp8_kernel<false>, grid, dim3(256), 0, s, A, lda, m, n, A8, ld8, A8T, ldT, scale, ntc,
                       flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ product

constexpr int KC8 = 128;   // one scale block of the contraction per iteration

template <int NB>
__global__ __launch_bounds__(256) void nn_fp8_kernel(const uint8_t* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ sA, int64_t s_row, int64_t s_k,
                                                     int64_t rows, int64_t K, const float* __restrict__ X,
                                                     int64_t ldx, int ncols, float* __restrict__ out, int64_t ldo,
                                                     int64_t part_stride, int64_t kchunk) {
  __shared__ u32x2 xs[NB * 4 * 64];   // (cb, t, lane) -> 8 E4M3 codes
  __shared__ float sxs[NB * 16];
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

  for (int64_t k0 = kbeg; k0 < kend; k0 += KC8) {
    // stage the X segment [k0, k0+128) of columns [cg0, cg0 + 16 NB): 16 threads per column, 8 values each
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = threadIdx.x + 256 * u;
      const int cl = it >> 4, ch = it & 15;
      const int c = cg0 + cl;
      const int64_t kk = k0 + 8 * ch;
      float v[8];
      if (c < ncols && kk + 8 <= kend) {
        const float* p = X + (int64_t)c * ldx + kk;
        const float4 q0 = *reinterpret_cast<const float4*>(p);
        const float4 q1 = *reinterpret_cast<const float4*>(p + 4);
        v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w; v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (c < ncols && kk + e < kend) ? X[(int64_t)c * ldx + kk + e] : 0.f;
      }
      float mx = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(v[e]));
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 16));
      const int ex = fp8_scale_exp(mx);
      uint32_t w0 = 0, w1 = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        w0 |= f32_to_e4m3(ldexpf(v[e], -ex)) << (8 * e);
        w1 |= f32_to_e4m3(ldexpf(v[4 + e], -ex)) << (8 * e);
      }
      const int cb = cl >> 4, cli = cl & 15, gg = ch >> 2, tt = ch & 3;
      xs[(cb * 4 + tt) * 64 + cli + 16 * gg] = u32x2{w0, w1};
      if (ch == 0) sxs[cl] = ldexpf(1.0f, ex);
    }
    // A: this lane's 32 contiguous codes of rows rbase + 16 rb + li
    u32x2 a[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t r = rbase + 16 * rb + li;
      if (r < rows) {
        const u32x4* p = reinterpret_cast<const u32x4*>(A + r * lda + k0 + 32 * g);
        const u32x4 q0 = p[0], q1 = p[1];
        a[rb][0] = u32x2{q0[0], q0[1]};
        a[rb][1] = u32x2{q0[2], q0[3]};
        a[rb][2] = u32x2{q1[0], q1[1]};
        a[rb][3] = u32x2{q1[2], q1[3]};
      } else {
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) a[rb][tt] = u32x2{0u, 0u};
      }
    }
    const float sa = sA[(int64_t)blockIdx.x * s_row + (k0 / KC8) * s_k];
    __syncthreads();
    f32x4 part[2][NB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) part[rb][cb] = M::zero();
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      long b[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) b[cb] = __builtin_bit_cast(long, xs[(cb * 4 + tt) * 64 + lane]);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const long av = __builtin_bit_cast(long, a[rb][tt]);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          part[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, b[cb], part[rb][cb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const float s = sa * sxs[cb * 16 + li];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[rb][cb][e] += s * part[rb][cb][e];
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

hipError_t launch_nn_fp8(const uint8_t* A, int64_t lda, const float* sA, int64_t s_row, int64_t s_k, int64_t rows,
                         int64_t K, const float* X, int64_t ldx, int ncols, float* out, int64_t ldo,
                         int64_t part_stride, int splits, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (lda % 128 != 0 || lda < K || (reinterpret_cast<uintptr_t>(A) & 15) != 0 || ldx % 4 != 0 ||
      (reinterpret_cast<uintptr_t>(X) & 15) != 0)
    return hipErrorInvalidValue;
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + KC8 - 1) / KC8 * KC8;
  if (kchunk < KC8) kchunk = KC8;
  const int used = (int)((K + kchunk - 1) / kchunk);
  int nb = (ncols + 15) / 16;
  nb = nb > 8 ? 8 : nb;
  const int groups = (ncols + nb * 16 - 1) / (nb * 16);
  dim3 grid((unsigned)((rows + 127) / 128), (unsigned)used, (unsigned)groups);
  switch (nb) {
#define RSVD_FP8_CASE(NBV)                                                                                   \
    case NBV: hipLaunchKernelGGL(nn_fp8_kernel<NBV>, grid, dim3(256), 0, s, A, lda, sA, s_row, s_k, rows, K, X, \
                                 ldx, ncols, out, ldo, part_stride, kchunk); break;
    RSVD_FP8_CASE(1) RSVD_FP8_CASE(2) RSVD_FP8_CASE(3) RSVD_FP8_CASE(4)
    RSVD_FP8_CASE(5) RSVD_FP8_CASE(6) RSVD_FP8_CASE(7) default: RSVD_FP8_CASE(8)
#undef RSVD_FP8_CASE
  }
  return hipGetLastError();
}

}  // namespace rsvd
