// Device-side helpers shared by the gfx950 kernels: MFMA wrappers, 4-wide
// vector loads/stores, wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

constexpr int kWave = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// One 16x16 MFMA tile with K = 4 per instruction.  Operand layout (both
// precisions): lane l supplies A(row l%16, k l/16) and B(k l/16, col l%16).
// Accumulator element r of lane l holds
//   f32: D(row 4*(l/16) + r, col l%16)
//   f64: D(row (l/16) + 4*r, col l%16)
// (measured on gfx950).  The kernels always want lane l to end up with four
// consecutive data rows 4*(l/16) + r, so the lane that supplies MFMA row i
// loads data row arow(i): the identity for f32, and the permutation
// i = g + 4e -> 4g + e for f64.
template <typename TC> struct Mma;
template <> struct Mma<float> {
  static __device__ __forceinline__ int arow(int i) { return i; }
  typedef f32x4 acc;
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<double> {
  static __device__ __forceinline__ int arow(int i) { return ((i & 3) << 2) | (i >> 2); }
  typedef f64x4 acc;
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T> struct V4 { T x[4]; };

template <typename T> __device__ __forceinline__ V4<T> v4_zero() {
  V4<T> v; v.x[0] = v.x[1] = v.x[2] = v.x[3] = T(0); return v;
}

// Aligned 4-element load (16 B for float, two 16 B loads for double).
__device__ __forceinline__ V4<float> v4_load(const float* p) {
  float4 t = *reinterpret_cast<const float4*>(p);
  V4<float> v; v.x[0] = t.x; v.x[1] = t.y; v.x[2] = t.z; v.x[3] = t.w; return v;
}
__device__ __forceinline__ V4<double> v4_load(const double* p) {
  double2 a = *reinterpret_cast<const double2*>(p);
  double2 b = *reinterpret_cast<const double2*>(p + 2);
  V4<double> v; v.x[0] = a.x; v.x[1] = a.y; v.x[2] = b.x; v.x[3] = b.y; return v;
}
__device__ __forceinline__ void v4_store(float* p, const V4<float>& v) {
  *reinterpret_cast<float4*>(p) = make_float4(v.x[0], v.x[1], v.x[2], v.x[3]);
}
__device__ __forceinline__ void v4_store(double* p, const V4<double>& v) {
  *reinterpret_cast<double2*>(p) = make_double2(v.x[0], v.x[1]);
  *reinterpret_cast<double2*>(p + 2) = make_double2(v.x[2], v.x[3]);
}

// Load elements [col, col+4) of row `row` of a row-major matrix with leading
// dimension ld; entries outside [0,rows) x [0,cols) read as zero.  The vector
// path is taken when VEC (caller guarantees ld % 4 == 0 and an aligned base)
// and the four entries are in range.
template <bool VEC, typename T>
__device__ __forceinline__ V4<T> load4_guarded(const T* base, int64_t ld, int64_t row, int64_t col,
                                               int64_t rows, int64_t cols) {
  if (row >= rows) return v4_zero<T>();
  const T* p = base + row * ld + col;
  if (VEC && col + 4 <= cols) return v4_load(p);
  V4<T> v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v.x[e] = (col + e < cols) ? p[e] : T(0);
  return v;
}

template <typename TD, typename TS>
__device__ __forceinline__ V4<TD> v4_cast(const V4<TS>& s) {
  V4<TD> d;
#pragma unroll
  for (int e = 0; e < 4; ++e) d.x[e] = static_cast<TD>(s.x[e]);
  return d;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace rsvd
