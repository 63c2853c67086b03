// Small helper kernels: flag reset (a fill kernel rather than a memset, so the
// sequence stays capturable in a HIP graph) and conversion of a caller-given
// row-major FP64 test matrix into the library's panel layout.
#include "internal.hpp"

namespace rsvd {

__global__ void fill_int_kernel(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// dst[c*ld_dst + r] = src[r*ld_src + c]
template <typename TO>
__global__ void rm_to_panel_kernel(const double* __restrict__ src, int64_t rows, int64_t cols, int64_t ld_src,
                                   TO* __restrict__ dst, int64_t ld_dst) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  int64_t r = t / cols, c = t % cols;
  dst[c * ld_dst + r] = static_cast<TO>(src[r * ld_src + c]);
}

template <typename TO>
hipError_t launch_rowmajor_to_panel(const double* src, int64_t rows, int64_t cols, int64_t ld_src, TO* dst,
                                    int64_t ld_dst, hipStream_t s) {
  int64_t work = rows * cols;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL((rm_to_panel_kernel<TO>), dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, src, rows,
                     cols, ld_src, dst, ld_dst);
  return hipGetLastError();
}

template hipError_t launch_rowmajor_to_panel<float>(const double*, int64_t, int64_t, int64_t, float*, int64_t,
                                                    hipStream_t);
template hipError_t launch_rowmajor_to_panel<double>(const double*, int64_t, int64_t, int64_t, double*, int64_t,
                                                     hipStream_t);

}  // namespace rsvd

namespace rsvd {

// Y[c*ldy + r] += alpha * X[c*ldx + r] for r < rows, c < ncols.
template <typename T>
__global__ void axpy_panel_kernel(T* __restrict__ Y, int64_t ldy, const T* __restrict__ X, int64_t ldx, int64_t rows,
                                  int ncols, T alpha) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * ncols) return;
  int64_t c = t / rows, r = t % rows;
  Y[c * ldy + r] += alpha * X[c * ldx + r];
}

template <typename T>
hipError_t launch_axpy_panel(T* Y, int64_t ldy, const T* X, int64_t ldx, int64_t rows, int ncols, T alpha,
                             hipStream_t s) {
  int64_t work = rows * ncols;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL((axpy_panel_kernel<T>), dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, Y, ldy, X, ldx,
                     rows, ncols, alpha);
  return hipGetLastError();
}

// norms[c] = || X[c*ld + 0 .. rows) ||_2, accumulated in FP64; one block per column.
template <typename T>
__global__ __launch_bounds__(256) void colnorm_kernel(const T* __restrict__ X, int64_t ld, int64_t rows,
                                                      double* __restrict__ norms) {
  __shared__ double red[4];
  const T* x = X + (int64_t)blockIdx.x * ld;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) {
    double v = (double)x[r];
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) norms[blockIdx.x] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

template <typename T>
hipError_t launch_colnorm(const T* X, int64_t ld, int64_t rows, int ncols, double* norms, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL((colnorm_kernel<T>), dim3((unsigned)ncols), dim3(256), 0, s, X, ld, rows, norms);
  return hipGetLastError();
}

// out[b] = sum of squares of rows [b*chunk, (b+1)*chunk) of A (m x n, lda), FP64.
template <typename T>
__global__ __launch_bounds__(256) void sumsq_rows_kernel(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                         int64_t chunk, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(m, r0 + chunk);
  for (int64_t r = r0; r < r1; ++r)
    for (int64_t c = threadIdx.x; c < n; c += 256) {
      double v = (double)A[r * lda + c];
      s += v * v;
    }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void sum_doubles_kernel(const double* __restrict__ in, int n, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += in[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// *out = ||A||_F^2 (FP64); partials: >= 1024 doubles of scratch.
template <typename T>
hipError_t launch_frob2(const T* A, int64_t lda, int64_t m, int64_t n, double* partials, double* out, hipStream_t s) {
  int64_t chunk = (m + 1023) / 1024;
  int nb = (int)((m + chunk - 1) / chunk);
  hipLaunchKernelGGL((sumsq_rows_kernel<T>), dim3((unsigned)nb), dim3(256), 0, s, A, lda, m, n, chunk, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_doubles_kernel, dim3(1), dim3(256), 0, s, partials, nb, out);
  return hipGetLastError();
}

template hipError_t launch_axpy_panel<float>(float*, int64_t, const float*, int64_t, int64_t, int, float, hipStream_t);
template hipError_t launch_axpy_panel<double>(double*, int64_t, const double*, int64_t, int64_t, int, double,
                                              hipStream_t);
template hipError_t launch_colnorm<float>(const float*, int64_t, int64_t, int, double*, hipStream_t);
template hipError_t launch_colnorm<double>(const double*, int64_t, int64_t, int, double*, hipStream_t);
template hipError_t launch_frob2<float>(const float*, int64_t, int64_t, int64_t, double*, double*, hipStream_t);
template hipError_t launch_frob2<double>(const double*, int64_t, int64_t, int64_t, double*, double*, hipStream_t);

// G <- (G + G^T) / 2 on the leading l x l block of a column-major matrix (ld ldg): one thread per pair
// (i, j), i <= j, so each entry is read before either of the pair is written.
__global__ void symmetrize_kernel(double* __restrict__ G, int64_t ldg, int l) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)l * l) return;
  const int i = (int)(t / l), j = (int)(t - (t / l) * l);
  if (i > j) return;
  const double v = 0.5 * (G[(int64_t)j * ldg + i] + G[(int64_t)i * ldg + j]);
  G[(int64_t)j * ldg + i] = v;
  G[(int64_t)i * ldg + j] = v;
}

hipError_t launch_symmetrize(double* G, int64_t ldg, int l, hipStream_t s) {
  const int64_t work = (int64_t)l * l;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, G, ldg, l);
  return hipGetLastError();
}

// out[i] = in[i]^2, i < n
__global__ void square_kernel(const double* __restrict__ in, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] * in[i];
}

hipError_t launch_square(const double* in, double* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(square_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace rsvd
