// The structured test matrix of Section 6 in real arithmetic and the sketch
// Y = A Omega in one pass over A.
//
// Section 6 replaces the Gaussian test matrix by Omega = D F S (a random
// diagonal, a fast unitary transform, a column subsampling), so that the
// sketch costs O(m n log l) instead of O(m n l).  All matrices here are real:
//   N = 2^p >= n (rows of A zero-padded to N), D = diag(d_i), d_i = +-1,
//   F = H_N / sqrt(N) with H_N(i, k) = (-1)^popcount(i & k) (Walsh-Hadamard),
//   S = l distinct columns s_0 .. s_{l-1} of the N x N identity,
//   Omega = the first n rows of D F S, so Y(r, j) = (H_N (d .* a_r))(s_j) / sqrt(N)
// for row a_r of A.  Random numbers: Philox4x32-10 under key = seed, stream
// 10: sign d_i is the lowest bit of word i mod 4 of counter (i div 4, 0, 10,
// 0); the subset is the first l steps of a Fisher-Yates shuffle of 0 .. N-1
// whose step j swaps perm[j] and perm[j + floor(u_j (N - j) / 2^32)], u_j
// = word j mod 4 of counter (j div 4, 1, 10, 0).
//
// Sketch kernel: one row at a time per workgroup, the sign-flipped row in LDS
// (one pad word per 32, so that every phase below reads and writes without
// bank conflicts).  The transform runs in radix-32 phases over 5 bits of the
// index each: a thread takes the 32 entries that differ in the phase's bits,
// runs the five butterfly stages in registers and writes them back.  The last
// phase is evaluated only at the l sampled indices (a signed sum of at most
// 32 entries each).  The next row's entries are loaded into registers while
// the current row is transformed (the barriers wait for LDS only, so those
// loads stay in flight).  HBM traffic: A once, the signs from L2, Y.
#include <math.h>

#include <algorithm>

#include "internal.hpp"
#include "philox.hpp"

namespace rsvd {

constexpr uint32_t kStreamSrht = 10;
constexpr int kSrhtThreads = 512;
constexpr int kSrhtMaxN = 32768;   // largest N: the FP32 row buffer (135 KB of LDS); 16384 for FP64

__device__ __forceinline__ int srht_phys(int i) { return i + (i >> 5); }

__device__ __forceinline__ void srht_lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((15) | (7 << 4) | (0 << 8) | (3 << 14));   // lgkmcnt(0) only
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Signs d_0 .. d_{n-1} and subset s_0 .. s_{l-1} (one workgroup).
template <typename T>
__global__ __launch_bounds__(kSrhtThreads) void srht_setup_kernel(uint64_t seed, int n, int N, int l,
                                                                  T* __restrict__ signs, int* __restrict__ subset) {
  __shared__ uint16_t perm[kSrhtMaxN];
  __shared__ uint32_t u[1024];
  static_assert(kSrhtThreads >= 64, "setup");
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int b = threadIdx.x; b < (n + 3) / 4; b += kSrhtThreads) {
    uint32_t c[4] = {(uint32_t)b, 0u, kStreamSrht, 0u};
    philox10(c, k0, k1);
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (4 * b + w < n) signs[4 * b + w] = (c[w] & 1u) ? T(-1) : T(1);
  }
  for (int b = threadIdx.x; b < (l + 3) / 4; b += kSrhtThreads) {
    uint32_t c[4] = {(uint32_t)b, 1u, kStreamSrht, 0u};
    philox10(c, k0, k1);
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (4 * b + w < l) u[4 * b + w] = c[w];
  }
  for (int i = threadIdx.x; i < N; i += kSrhtThreads) perm[i] = (uint16_t)i;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < l; ++j) {
      const int r = j + (int)(((uint64_t)u[j] * (uint64_t)(N - j)) >> 32);
      const uint16_t t = perm[j];
      perm[j] = perm[r];
      perm[r] = t;
      subset[j] = perm[j];
    }
  }
}

// One full radix-32 phase over bits SH .. SH+4 of the index (SH = 0 or 5: the only places a full phase
// falls for N <= 2^15, the last phase being taken at the outputs).  Group g holds the 32 entries that
// differ in those bits; with the padded index i + i / 32 their LDS positions are q(g) + s (SH = 0) or
// q(g) + 33 s (SH = 5), so every access has a compile-time offset.
template <int SH, typename T, int THR>
__device__ __forceinline__ void srht_phase(T* __restrict__ x, int N, int tid) {
  constexpr int STEP = SH == 0 ? 1 : 33;
  for (int g = tid; g < (N >> 5); g += THR) {
    const int q = SH == 0 ? 33 * g : (g & 31) + ((g >> 5) << 10) + ((g >> 5) << 5);
    T v[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) v[s] = x[q + STEP * s];
#pragma unroll
    for (int h = 1; h < 32; h <<= 1)
#pragma unroll
      for (int s = 0; s < 32; ++s)
        if ((s & h) == 0) {
          const T a0 = v[s], b0 = v[s + h];
          v[s] = a0 + b0;
          v[s + h] = a0 - b0;
        }
#pragma unroll
    for (int s = 0; s < 32; ++s) x[q + STEP * s] = v[s];
  }
}

// Output of one sampled column s: sum over t < 2^nb of (-1)^popcount(t & (s >> sh)) x(base + t 2^sh), base
// the low sh bits of s; lane jq of the column's four takes the terms t = jq tq .. jq tq + tq - 1 (tq <= 8).
template <typename T>
__device__ __forceinline__ T srht_out_part(const T* __restrict__ x, int s, int sh, int nt, int tq, int jq) {
  const int hi = s >> sh, base = s & ((1 << sh) - 1);
  T v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int t = jq * tq + u;
    const int i = base + (t << sh);
    v[u] = (u < tq && t < nt) ? x[i + (i >> 5)] : T(0);
  }
  T acc = T(0);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int t = jq * tq + u;
    acc += (__popc((unsigned)(t & hi)) & 1) ? -v[u] : v[u];
  }
  return acc;
}

// out(r, j) = (H_N (d .* a_r))(s_j) * scale, written at out[r * osr + j * osc].  VW entries of a row per
// load (VW = 16 bytes / sizeof(T) when A and lda allow aligned 16-byte loads, 1 otherwise); consecutive
// lanes load consecutive 16-byte pieces of the row.
template <typename T, int VW>
__global__ __launch_bounds__(kSrhtThreads) void srht_sketch_kernel(const T* __restrict__ A, int64_t lda, int64_t m,
                                                                   int n, int p, const T* __restrict__ signs,
                                                                   const int* __restrict__ subset, int l, T scale,
                                                                   T* __restrict__ out, int64_t osr, int64_t osc) {
  extern __shared__ __align__(16) unsigned char srht_lds[];
  T* x = reinterpret_cast<T*>(srht_lds);   // at least VW kSrhtThreads entries (padded): row stores need no bound
  const int N = 1 << p;
  const int nph = p == 0 ? 1 : (p + 4) / 5;   // phases of 5 bits; the last one is taken at the outputs only
  const int tid = threadIdx.x;
  constexpr int CH = VW * kSrhtThreads;                                     // row entries per load round
  constexpr int NG = (sizeof(T) == 8 ? kSrhtMaxN / 2 : kSrhtMaxN) / CH;    // load rounds at the largest N
  // group e of a thread holds row entries VW (tid + kSrhtThreads e) + c, c < VW.  Groups e < efull exist
  // whole for every thread, group efull in part (uniform bounds keep the per-group conditions scalar).
  const int efull = n / CH;
  const int rem = n - efull * CH - VW * tid;   // entries of group efull this thread holds (may be <= 0)
  const int en = (N + CH - 1) / CH;            // groups the padded row holds
  struct Vec { T v[VW]; };
  auto load = [&](const T* a, int e) {
    Vec r;
    const T* q = a + VW * (tid + kSrhtThreads * e);
    if (e < efull) {
      if constexpr (VW == 4) {
        const float4 t = *reinterpret_cast<const float4*>(q);
        r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
      } else if constexpr (VW == 2) {
        const double2 t = *reinterpret_cast<const double2*>(q);
        r.v[0] = t.x; r.v[1] = t.y;
      } else {
        r.v[0] = q[0];
      }
    } else {
#pragma unroll
      for (int c = 0; c < VW; ++c) r.v[c] = (e == efull && c < rem) ? q[c] : T(0);
    }
    return r;
  };
  uint64_t neg = 0;   // bit VW e + c: the sign of entry c of group e is -1
  {
    Vec sg[NG];
#pragma unroll
    for (int e = 0; e < NG; ++e) sg[e] = load(signs, e);
#pragma unroll
    for (int e = 0; e < NG; ++e)
#pragma unroll
      for (int c = 0; c < VW; ++c)
        if (sg[e].v[c] < T(0)) neg |= 1ull << (VW * e + c);
  }
  Vec nx[NG];
  auto fetch = [&](int64_t r) {
    const T* a = A + min(r, m - 1) * lda;
#pragma unroll
    for (int e = 0; e < NG; ++e) nx[e] = load(a, e);
  };
  // output phase: four lanes per sampled column, each summing a quarter of its (at most 32) signed terms
  const int sh = 5 * (nph - 1), nb = p - sh;
  const int nt = 1 << nb, tq = (nt + 3) / 4;
  const int jq = tid & 3;
  const int s0 = subset[min(tid >> 2, l - 1)];   // the first block of sampled columns, read once
  fetch(blockIdx.x);
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
#pragma unroll
    for (int e = 0; e < NG; ++e) {
      if (e < en) {
#pragma unroll
        for (int c = 0; c < VW; ++c) {
          const int i = VW * (tid + kSrhtThreads * e) + c;
          x[i + (i >> 5)] = ((neg >> (VW * e + c)) & 1ull) ? -nx[e].v[c] : nx[e].v[c];
        }
      }
    }
    srht_lds_barrier();
    fetch(r + gridDim.x);   // the next row, in flight during the transform
    if (nph >= 2) {
      srht_phase<0, T, kSrhtThreads>(x, N, tid);
      srht_lds_barrier();
    }
    if (nph >= 3) {
      srht_phase<5, T, kSrhtThreads>(x, N, tid);
      srht_lds_barrier();
    }
    for (int j0 = 0; j0 < l; j0 += kSrhtThreads / 4) {
      const int j = j0 + (tid >> 2);
      const int s = j0 == 0 ? s0 : subset[min(j, l - 1)];
      T acc = srht_out_part(x, s, sh, nt, tq, jq);
      acc += __shfl_xor(acc, 1, 4);
      acc += __shfl_xor(acc, 2, 4);
      if (jq == 0 && j < l) out[r * osr + (int64_t)j * osc] = acc * scale;
    }
    srht_lds_barrier();
  }
}

int srht_max_n(int es) { return es == 8 ? kSrhtMaxN / 2 : kSrhtMaxN; }

template <typename T>
hipError_t launch_srht_setup(uint64_t seed, int n, int l, T* signs, int* subset, hipStream_t s) {
  if (n < 1 || n > srht_max_n(sizeof(T)) || l < 1 || l > 1024) return hipErrorInvalidValue;
  int p = 0;
  while ((1 << p) < n) ++p;
  if (l > (1 << p)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((srht_setup_kernel<T>), dim3(1), dim3(kSrhtThreads), 0, s, seed, n, 1 << p, l, signs, subset);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_srht_sketch(const T* A, int64_t lda, int64_t m, int n, const T* signs, const int* subset, int l,
                              T* out, int64_t osr, int64_t osc, hipStream_t s) {
  if (m < 1) return hipSuccess;
  if (n < 1 || n > srht_max_n(sizeof(T)) || lda < n || l < 1) return hipErrorInvalidValue;
  int p = 0;
  while ((1 << p) < n) ++p;
  const int N = 1 << p;
  if (l > N) return hipErrorInvalidValue;
  constexpr int VW = 16 / sizeof(T);
  const bool vec = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda * (int64_t)sizeof(T)) % 16 == 0 &&
                   (reinterpret_cast<uintptr_t>(signs) & 15) == 0;
  const int Nb = std::max(N, (vec ? VW : 1) * kSrhtThreads);   // the row buffer covers one load round at least
  const size_t sh = (size_t)(Nb + Nb / 32 + 1) * sizeof(T);
  static bool attr_set[2][2] = {{false, false}, {false, false}};
  const int ti = sizeof(T) == 8 ? 1 : 0;
  const void* fn = vec ? reinterpret_cast<const void*>(&srht_sketch_kernel<T, VW>)
                       : reinterpret_cast<const void*>(&srht_sketch_kernel<T, 1>);
  if (!attr_set[ti][vec]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((kSrhtMaxN + kSrhtMaxN / 32 + 1) * sizeof(float)));
    if (e != hipSuccess) return e;
    attr_set[ti][vec] = true;
  }
  int dev = 0, cu = 256;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cu = prop.multiProcessorCount;
  // LDS per workgroup sets the occupancy: one row buffer of 135 KB at the largest N, so one per compute unit;
  // small rows fit two
  const int per_cu = sh <= 72 * 1024 ? 2 : 1;
  const int64_t grid = std::min<int64_t>(m, (int64_t)cu * per_cu);
  const T scale = (T)(1.0 / sqrt((double)N));
  if (vec)
    hipLaunchKernelGGL((srht_sketch_kernel<T, VW>), dim3((unsigned)grid), dim3(kSrhtThreads), sh, s, A, lda, m, n,
                       p, signs, subset, l, scale, out, osr, osc);
  else
    hipLaunchKernelGGL((srht_sketch_kernel<T, 1>), dim3((unsigned)grid), dim3(kSrhtThreads), sh, s, A, lda, m, n, p,
                       signs, subset, l, scale, out, osr, osc);
  return hipGetLastError();
}

template hipError_t launch_srht_setup<float>(uint64_t, int, int, float*, int*, hipStream_t);
template hipError_t launch_srht_setup<double>(uint64_t, int, int, double*, int*, hipStream_t);
template hipError_t launch_srht_sketch<float>(const float*, int64_t, int64_t, int, const float*, const int*, int,
                                              float*, int64_t, int64_t, hipStream_t);
template hipError_t launch_srht_sketch<double>(const double*, int64_t, int64_t, int, const double*, const int*, int,
                                               double*, int64_t, int64_t, hipStream_t);

}  // namespace rsvd
