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
