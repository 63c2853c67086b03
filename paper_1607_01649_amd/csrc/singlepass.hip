// Small dense FP64 steps of the single-pass factorisations (Section 5): the
// k x k core C is the least-squares solution of the joint system
//   M1 C = N1,  C M2 = N2          (general matrices, Section 5.2)
// or of C M = N over symmetric C   (symmetric matrices, Section 5.1).
// Setting the gradient of the summed squared residuals to zero gives a
// Sylvester equation P1 C + C P2 = S with P1 = M1^T M1, P2 = M2 M2^T and
// S = M1^T N1 + N2 M2^T (symmetric case: P1 = P2 = M M^T, S = N M^T + M N^T).
// With the eigendecompositions P1 = Z1 diag(a) Z1^T and P2 = Z2 diag(b) Z2^T
// (both positive semidefinite) it decouples entry by entry:
//   C = Z1 [ (Z1^T S Z2)_ij / (a_i + b_j) ] Z2^T.
// The eigendecompositions come from the one-sided Jacobi kernel; this file
// holds the small products and the entrywise steps, all in FP64 (k <= 1024,
// column-major matrices with leading dimensions that are multiples of 16).
#include "internal.hpp"

namespace rsvd {

namespace {

constexpr int kSgTile = 32;   // output tile of the small product (32 x 32, 256 threads, 2 x 2 per thread)
constexpr int kSgK = 16;      // contraction chunk staged in LDS

template <typename TO>
__global__ __launch_bounds__(256) void small_gemm_kernel(int M, int N, int K, const double* __restrict__ A,
                                                         int64_t lda, int ta, const double* __restrict__ B,
                                                         int64_t ldb, int tb, TO* __restrict__ out, int64_t ldo,
                                                         int acc, const double* __restrict__ inv_scale) {
  __shared__ double As[kSgK][kSgTile + 1];   // As[kk][i] = op(A)(i0 + i, k0 + kk)
  __shared__ double Bs[kSgK][kSgTile + 1];   // Bs[kk][j] = op(B)(k0 + kk, j0 + j)
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.x * kSgTile, j0 = blockIdx.y * kSgTile;
  double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
  for (int k0 = 0; k0 < K; k0 += kSgK) {
    for (int e = threadIdx.x; e < kSgTile * kSgK; e += 256) {
      const int r = e & (kSgTile - 1), kk = e >> 5;
      const int gk = k0 + kk;
      const int gi = i0 + r, gj = j0 + r;
      double a = 0.0, b = 0.0;
      if (gi < M && gk < K) a = ta ? A[(int64_t)gi * lda + gk] : A[(int64_t)gk * lda + gi];
      if (gj < N && gk < K) b = tb ? B[(int64_t)gk * ldb + gj] : B[(int64_t)gj * ldb + gk];
      As[kk][r] = a;
      Bs[kk][r] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kSgK; ++kk) {
      const double a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const double b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
      c00 = fma(a0, b0, c00);
      c01 = fma(a0, b1, c01);
      c10 = fma(a1, b0, c10);
      c11 = fma(a1, b1, c11);
    }
    __syncthreads();
  }
  const double cv[2][2] = {{c00, c01}, {c10, c11}};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = i0 + ty + 16 * a, j = j0 + tx + 16 * b;
      if (i >= M || j >= N) continue;
      double v = cv[a][b];
      if (inv_scale) {
        const double s = inv_scale[j];
        v = s > 0.0 ? v / s : 0.0;
      }
      TO* o = out + (int64_t)j * ldo + i;
      *o = static_cast<TO>(acc ? static_cast<double>(*o) + v : v);
    }
}

// X(i, j) <- X(i, j) / (a_i + b_j); entries whose denominator is at or below cut_rel (a_0 + b_0) (a, b
// descending, so a_0 + b_0 is the largest) are set to zero: the minimum-norm solution along directions in
// which neither equation set determines C.
__global__ __launch_bounds__(256) void sylv_divide_kernel(double* __restrict__ X, int64_t ldx, int k1, int k2,
                                                          const double* __restrict__ a, const double* __restrict__ b,
                                                          double cut_rel) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)k1 * k2) return;
  const int i = (int)(idx % k1), j = (int)(idx / k1);
  const double den = a[i] + b[j];
  const double cut = cut_rel * (a[0] + b[0]);
  double* x = X + (int64_t)j * ldx + i;
  *x = den > cut ? *x / den : 0.0;
}

// out[j] = sum_r X(r, j) Y(r, j), one wave per column.
__global__ __launch_bounds__(256) void coldot_kernel(const double* __restrict__ X, const double* __restrict__ Y,
                                                     int64_t ld, int rows, int ncols, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= ncols) return;
  double s = 0.0;
  for (int r = lane; r < rows; r += 64) s = fma(X[(int64_t)j * ld + r], Y[(int64_t)j * ld + r], s);
  s = wave_sum(s);
  if (lane == 0) out[j] = s;
}

// out(j, i) = in(i, j) for an rows x cols matrix (column-major, leading dimensions ldi, ldo).
__global__ __launch_bounds__(256) void transpose64_kernel(const double* __restrict__ in, int64_t ldi, int rows,
                                                          int cols, double* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)rows * cols) return;
  const int i = (int)(idx % rows), j = (int)(idx / rows);
  out[(int64_t)i * ldo + j] = in[(int64_t)j * ldi + i];
}

// x <- the bfloat16 value nearest to x (ties to even), kept in binary32: a test matrix drawn for a bf16
// sketch, so that the least-squares equations use the matrix the sketch was formed with.
__global__ __launch_bounds__(256) void round_bf16_kernel(float* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t u = __float_as_uint(x[i]);
  u += 0x7FFFu + ((u >> 16) & 1u);
  x[i] = __uint_as_float(u & 0xFFFF0000u);
}

}  // namespace

hipError_t launch_round_bf16(float* x, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(round_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

hipError_t launch_transpose64(const double* in, int64_t ldi, int rows, int cols, double* out, int64_t ldo,
                              hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, ldi, rows, cols,
                     out, ldo);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_small_gemm(int M, int N, int K, const double* A, int64_t lda, bool ta, const double* B, int64_t ldb,
                             bool tb, TO* out, int64_t ldo, bool acc, const double* inv_scale, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + kSgTile - 1) / kSgTile), (unsigned)((N + kSgTile - 1) / kSgTile));
  hipLaunchKernelGGL((small_gemm_kernel<TO>), grid, dim3(256), 0, s, M, N, K, A, lda, ta ? 1 : 0, B, ldb,
                     tb ? 1 : 0, out, ldo, acc ? 1 : 0, inv_scale);
  return hipGetLastError();
}
template hipError_t launch_small_gemm<double>(int, int, int, const double*, int64_t, bool, const double*, int64_t,
                                              bool, double*, int64_t, bool, const double*, hipStream_t);
template hipError_t launch_small_gemm<float>(int, int, int, const double*, int64_t, bool, const double*, int64_t,
                                             bool, float*, int64_t, bool, const double*, hipStream_t);

hipError_t launch_sylv_divide(double* X, int64_t ldx, int k1, int k2, const double* a, const double* b,
                              double cut_rel, hipStream_t s) {
  const int64_t n = (int64_t)k1 * k2;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sylv_divide_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, ldx, k1, k2, a, b,
                     cut_rel);
  return hipGetLastError();
}

hipError_t launch_coldot(const double* X, const double* Y, int64_t ld, int rows, int ncols, double* out,
                         hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(coldot_kernel, dim3((unsigned)((ncols + 3) / 4)), dim3(256), 0, s, X, Y, ld, rows, ncols, out);
  return hipGetLastError();
}

}  // namespace rsvd
