// Gaussian test matrices on the device: Philox4x32-10 (Salmon, Moraes, Dror,
// Shaw, SC'11) and the Box-Muller transform.  Entry (i, j) of the family
// (seed, stream) depends on (seed, stream, i, j) only, so a matrix can be
// extended by further columns later (the blocked range finder of Figure 12
// draws its blocks as the continuation of Omega).
#include "internal.hpp"
#include "philox.hpp"

namespace rsvd {

__global__ void philox_kernel(int64_t count, const uint32_t* __restrict__ ctr, uint32_t k0, uint32_t k1,
                              uint32_t* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  philox10(c, k0, k1);
  out[4 * i] = c[0]; out[4 * i + 1] = c[1]; out[4 * i + 2] = c[2]; out[4 * i + 3] = c[3];
}

// Two standard normals from one Philox call: rows 2*i2 (cos) and 2*i2+1 (sin).
__device__ __forceinline__ void gauss_pair(uint64_t seed, uint32_t stream, uint32_t i2, uint32_t col,
                                           double& z0, double& z1) {
  uint32_t c[4] = {i2, col, stream, 0u};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  uint64_t v1 = ((((uint64_t)c[0]) << 32) | c[1]) >> 11;
  uint64_t v2 = ((((uint64_t)c[2]) << 32) | c[3]) >> 11;
  const double s53 = 1.1102230246251565404e-16;   // 2^-53
  double u1 = ((double)v1 + 0.5) * s53;
  double u2 = ((double)v2 + 0.5) * s53;
  double rad = sqrt(-2.0 * log(u1));
  double th = 6.283185307179586477 * u2;           // 2 pi, rounded to binary64
  z0 = rad * cos(th);
  z1 = rad * sin(th);
}

// out(row, c) for row < rows, c < cols, with the element written at
// out[c * col_stride + row * row_stride]: covers row-major (row_stride = ld,
// col_stride = 1) and the library's column-panel layout (row_stride = 1,
// col_stride = ld).  One thread per (row pair, column).
template <typename T>
__global__ void gaussian_kernel(uint64_t seed, uint32_t stream, int64_t rows, int64_t cols, int64_t col0,
                                T* __restrict__ out, int64_t row_stride, int64_t col_stride) {
  int64_t pairs = (rows + 1) / 2;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= pairs * cols) return;
  int64_t i2 = t % pairs, c = t / pairs;
  double z0, z1;
  gauss_pair(seed, stream, (uint32_t)i2, (uint32_t)(col0 + c), z0, z1);
  int64_t r0 = 2 * i2;
  out[c * col_stride + r0 * row_stride] = (T)z0;
  if (r0 + 1 < rows) out[c * col_stride + (r0 + 1) * row_stride] = (T)z1;
}

hipError_t launch_philox(int64_t count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, ctr, k0, k1, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gaussian(uint64_t seed, uint32_t stream, int64_t rows, int64_t cols, int64_t col0, T* out,
                           int64_t row_stride, int64_t col_stride, hipStream_t s) {
  int64_t work = ((rows + 1) / 2) * cols;
  if (work <= 0) return hipSuccess;
  int64_t blocks = (work + 255) / 256;
  hipLaunchKernelGGL(gaussian_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, seed, stream, rows, cols,
                     col0, out, row_stride, col_stride);
  return hipGetLastError();
}

template hipError_t launch_gaussian<float>(uint64_t, uint32_t, int64_t, int64_t, int64_t, float*, int64_t,
                                           int64_t, hipStream_t);
template hipError_t launch_gaussian<double>(uint64_t, uint32_t, int64_t, int64_t, int64_t, double*, int64_t,
                                            int64_t, hipStream_t);

}  // namespace rsvd
