// Partial column-pivoted QR and the interpolative decomposition built on it
// (Sections 10-11), for a short wide matrix held as the rows of a panel: the
// columns y_c (c < N) of the l x N matrix are the rows of an N x l panel Y
// (y_c[t] = Y[t * ld + c]), which is how the library holds its sketches.
//
// Pivoted Gram-Schmidt, left-looking: after j steps, with q_0 .. q_{j-1}
// orthonormal and S = Q^T Y, the residual norm of column c is ||y_c||^2 -
// sum_i S(i, c)^2.  Step j:
//   - every column: S(j, c) = q_j . y_c, norm downdated (recomputed from the
//     residual when the downdate has lost more than half the digits, as in
//     LAPACK's column-pivoted QR), and the block's largest residual;
//   - the last block to finish (a ticket counter; no block ever waits) picks
//     the next pivot p (largest residual, lowest index on ties) and forms
//     q_{j+1} from y_p by Gram-Schmidt twice.
// One launch per step; the panel is read once per step (it stays in the
// last-level cache for the sizes of a sketch): a block takes 256 columns, a
// quarter of its threads a quarter of the rows each, every value of a
// thread's share loaded before any is used, so that the step is bound by the
// panel's bandwidth rather than by a chain of load latencies.
//
// The column ID then needs Z = S11^-1 S with S11 = S(:, J) upper triangular
// (Z(:, J) = I, Z elsewhere T = S11^-1 S12): one thread per column runs the
// back substitution, its partial solution in LDS.
#include <float.h>

#include "internal.hpp"

namespace rsvd {

namespace {

constexpr int kCpThreads = 1024;    // threads per block of the step kernel
constexpr int kCpCols = 256;        // columns per block: 256 threads per quarter of the rows
constexpr int kCpGroups = kCpThreads / kCpCols;
constexpr int kCpMaxL = 128;        // rows of the short wide matrix
constexpr int kCpRows = kCpMaxL / kCpGroups;   // rows per wave at most
constexpr int kSolveThreads = 64;   // columns per block of the triangular solve

// Block argmax of (v, c): the larger value, the lower index on ties; invalid entries carry v = -1.
__device__ void block_argmax(double& v, int& c, double* sv, int* sc) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oc = __shfl_xor(c, o, 64);
    if (ov > v || (ov == v && oc >= 0 && (c < 0 || oc < c))) { v = ov; c = oc; }
  }
  if ((tid & 63) == 0) { sv[tid >> 6] = v; sc[tid >> 6] = c; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kCpThreads / 64; ++w)
      if (sv[w] > v || (sv[w] == v && sc[w] >= 0 && (c < 0 || sc[w] < c))) { v = sv[w]; c = sc[w]; }
  }
}

// Work of the last block of a step: pick the pivot among the block maxima, form q_{j1} (j1 = index of the new
// vector) from y_p by two projections against q_0 .. q_{j1-1} (the first uses S(:, p)), record the pivot.
template <typename T>
__device__ void elect_and_build(const T* __restrict__ Y, int64_t ld, int l, int j1, int nblk,
                                const double* __restrict__ blkmax, const int* __restrict__ blkidx, double* Q, int LQ,
                                const double* S, int64_t ldS, double* nrm2, int* J, double* sv, int* sc) {
  const int tid = threadIdx.x;
  __shared__ double vsh[kCpMaxL];
  __shared__ double wsh[kCpMaxL];
  __shared__ double part[kCpThreads];
  __shared__ int piv;
  double v = -1.0;
  int c = -1;
  for (int b = tid; b < nblk; b += kCpThreads) {
    const double bv = blkmax[b];
    const int bc = blkidx[b];
    if (bv > v || (bv == v && bc >= 0 && (c < 0 || bc < c))) { v = bv; c = bc; }
  }
  block_argmax(v, c, sv, sc);
  if (tid == 0) piv = c;
  __syncthreads();
  const int p = piv;
  if (p < 0) return;   // no column left (cannot happen for j1 < min(l, N))
  // Q has j1 vectors of l entries (Q(i, t) at Q[i*LQ + t], L2-resident).  The sums over i below take thread
  // (t = tid % 128, part h = tid / 128) over one of kNh contiguous ranges of i, unrolled so that its loads are
  // in flight together, and add the parts in order; Q^T v takes one wave per vector.
  constexpr int kNh = kCpThreads / 128;
  const int t = tid & 127, h = tid >> 7;
  const int ib = j1 * h / kNh, ie = j1 * (h + 1) / kNh;
  auto q_times = [&](const double* coef) {   // part[tid] = sum over this thread's i of Q(i, t) coef[i]
    double a = 0.0;
    if (t < l) {
#pragma unroll 8
      for (int i = ib; i < ie; ++i) a = fma(Q[(int64_t)i * LQ + t], coef[i], a);
    }
    part[tid] = a;
  };
  // first projection: v = y_p - Q S(:, p)
  if (tid < j1) wsh[tid] = S[(int64_t)tid * ldS + p];
  __syncthreads();
  q_times(wsh);
  __syncthreads();
  auto part_sum = [&]() {
    double a = 0.0;
#pragma unroll
    for (int hh = 0; hh < kNh; ++hh) a += part[tid + 128 * hh];
    return a;
  };
  if (tid < l) vsh[tid] = static_cast<double>(Y[(int64_t)tid * ld + p]) - part_sum();
  __syncthreads();
  // second projection: w = Q^T v, v -= Q w
  {
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll 4
    for (int i = wv; i < j1; i += kCpThreads / 64) {
      double a = 0.0;
      if (lane < l) a = Q[(int64_t)i * LQ + lane] * vsh[lane];
      if (lane + 64 < l) a = fma(Q[(int64_t)i * LQ + lane + 64], vsh[lane + 64], a);
      a = wave_sum(a);
      if (lane == 0) wsh[i] = a;
    }
  }
  __syncthreads();
  q_times(wsh);
  __syncthreads();
  double x = 0.0;
  if (tid < l) x = vsh[tid] - part_sum();
  double ss = wave_sum(x * x);
  if ((tid & 63) == 0) sv[tid >> 6] = ss;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < kCpThreads / 64; ++w) tot += sv[w];
  const double inv = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
  if (tid < LQ) Q[(int64_t)j1 * LQ + tid] = tid < l ? x * inv : 0.0;
  if (tid == 0) {
    J[j1] = p;
    nrm2[p] = -1.0;   // chosen: no longer a candidate
  }
}

// Rows [r0, r0 + nr) of column c (nr <= kCpRows), all loaded before any is used, so that a wave has its
// whole share of the column in flight at once; rows past the end read as zero.
template <typename T>
__device__ __forceinline__ void load_rows(const T* __restrict__ Y, int64_t ld, int64_t c, bool valid, int r0, int nr,
                                          double (&y)[kCpRows]) {
#pragma unroll
  for (int u = 0; u < kCpRows; ++u) y[u] = (valid && u < nr) ? static_cast<double>(Y[(int64_t)(r0 + u) * ld + c]) : 0.0;
}

// The four waves' partial sums of a column, added in wave order; returned to every thread of the column.
__device__ __forceinline__ double column_sum(double v, double* red) {
  const int lane = threadIdx.x & (kCpCols - 1), grp = threadIdx.x / kCpCols;
  red[grp * kCpCols + lane] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int g = 0; g < kCpGroups; ++g) t += red[g * kCpCols + lane];
  __syncthreads();
  return t;
}

// Norms of every column and the first pivot.  Block b holds columns 256 b .. 256 b + 255 (thread tid: column
// tid % 256) and threads [256 g, 256 g + 256) rows [g R, g R + R), R = ceil(l / 4).  One block per compute
// unit at the sizes of a sketch: the election's ticket counter takes one atomic per block.
template <typename T>
__global__ __launch_bounds__(kCpThreads) void cpqr_init_kernel(const T* __restrict__ Y, int64_t ld, int64_t N, int l,
                                                               double* Q, int LQ, const double* S, int64_t ldS,
                                                               double* nrm2, double* orig, double* blkmax,
                                                               int* blkidx, unsigned* counter, int* J) {
  __shared__ double sv[kCpThreads / 64];
  __shared__ int sc[kCpThreads / 64];
  __shared__ double red[kCpThreads];
  __shared__ bool last;
  const int lane = threadIdx.x & (kCpCols - 1), grp = threadIdx.x / kCpCols;
  const int64_t c = (int64_t)blockIdx.x * kCpCols + lane;
  const int R = (l + kCpGroups - 1) / kCpGroups;
  const int r0 = grp * R, nr = max(0, min(R, l - r0));
  double y[kCpRows];
  load_rows<T>(Y, ld, c, c < N, r0, nr, y);
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < kCpRows; ++u) part = fma(y[u], y[u], part);
  const double s = column_sum(part, red);
  double v = -1.0;
  int ci = -1;
  if (grp == 0 && c < N) {
    nrm2[c] = s;
    orig[c] = s;
    v = s;
    ci = (int)c;
  }
  block_argmax(v, ci, sv, sc);
  if (threadIdx.x == 0) {
    blkmax[blockIdx.x] = v;
    blkidx[blockIdx.x] = ci;
    __threadfence();
    last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  elect_and_build<T>(Y, ld, l, 0, gridDim.x, blkmax, blkidx, Q, LQ, S, ldS, nrm2, J, sv, sc);
  if (threadIdx.x == 0) *counter = 0u;
}

// Step j: row j of S, downdated norms, and (when another step follows) the next pivot and q_{j+1}.  Layout as
// the init kernel.
template <typename T>
__global__ __launch_bounds__(kCpThreads) void cpqr_step_kernel(const T* __restrict__ Y, int64_t ld, int64_t N, int l,
                                                               int j, int k, double* Q, int LQ, double* S,
                                                               int64_t ldS, double* nrm2, const double* orig,
                                                               double* blkmax, int* blkidx, unsigned* counter,
                                                               int* J) {
  __shared__ double qs[kCpMaxL];
  __shared__ double sv[kCpThreads / 64];
  __shared__ int sc[kCpThreads / 64];
  __shared__ double red[kCpThreads];
  __shared__ int recompute;   // some column of the block takes the norm recomputation
  __shared__ bool last;
  const int tid = threadIdx.x;
  const int lane = tid & (kCpCols - 1), grp = tid / kCpCols;
  const int64_t c = (int64_t)blockIdx.x * kCpCols + lane;
  const bool valid = c < N;
  const int R = (l + kCpGroups - 1) / kCpGroups;
  const int r0 = grp * R, nr = max(0, min(R, l - r0));
  double y[kCpRows];
  load_rows<T>(Y, ld, c, valid, r0, nr, y);
  if (tid < l) qs[tid] = Q[(int64_t)j * LQ + tid];
  if (tid == 0) recompute = 0;
  __syncthreads();
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < kCpRows; ++u)
    if (u < nr) part = fma(qs[r0 + u], y[u], part);
  const double s = column_sum(part, red);
  if (grp == 0 && valid) S[(int64_t)j * ldS + c] = s;
  if (j + 1 >= k) return;   // uniform: the last step elects no pivot, its norms are not needed
  // downdated norm; LAPACK's safeguard recomputes it from the residual once it is below sqrt(eps) of the
  // original norm squared (every wave its rows, summed as above)
  double r = valid ? nrm2[c] : -1.0;
  const bool cand = r >= 0.0;
  if (cand) r -= s * s;
  const bool redo = cand && r <= 1.4901161193847656e-08 * orig[c];
  if (redo && grp == 0) recompute = 1;
  __syncthreads();
  if (recompute) {   // uniform
    double rp = 0.0;
    if (redo) {
#pragma unroll
      for (int u = 0; u < kCpRows; ++u) {
        if (u < nr) {
          double x = y[u];
          for (int i = 0; i <= j; ++i) x -= Q[(int64_t)i * LQ + r0 + u] * S[(int64_t)i * ldS + c];
          rp = fma(x, x, rp);
        }
      }
    }
    const double rr = column_sum(rp, red);
    if (redo) r = rr;
  }
  double v = -1.0;
  int ci = -1;
  if (grp == 0 && cand) {
    nrm2[c] = r;
    v = r;
    ci = (int)c;
  }
  block_argmax(v, ci, sv, sc);
  if (tid == 0) {
    blkmax[blockIdx.x] = v;
    blkidx[blockIdx.x] = ci;
    __threadfence();
    last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  elect_and_build<T>(Y, ld, l, j + 1, gridDim.x, blkmax, blkidx, Q, LQ, S, ldS, nrm2, J, sv, sc);
  if (tid == 0) *counter = 0u;
}

// S11(i, t) = S(i, J[t]) (k x k, column-major, leading dimension LK).
__global__ __launch_bounds__(256) void cpqr_s11_kernel(const double* __restrict__ S, int64_t ldS, int k,
                                                       const int* __restrict__ J, double* __restrict__ S11, int LK) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= k * k) return;
  const int i = idx % k, t = idx / k;
  S11[(int64_t)t * LK + i] = S[(int64_t)i * ldS + J[t]];
}

// Z(:, c) = S11^-1 S(:, c) by back substitution, one thread per column; Z (k x N, row i at Z + i * ldZ) and/or
// X = Z^T (N x k row-major, leading dimension ldx).
template <typename TX>
__global__ __launch_bounds__(kSolveThreads) void id_solve_kernel(const double* __restrict__ S, int64_t ldS, int64_t N,
                                                                 int k, const double* __restrict__ S11, int LK,
                                                                 double* __restrict__ Z, int64_t ldZ,
                                                                 TX* __restrict__ X, int64_t ldx) {
  extern __shared__ double xs[];   // xs[i * kSolveThreads + lane]
  const int lane = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * kSolveThreads + lane;
  const bool ok = c < N;
  for (int i = k - 1; i >= 0; --i) {
    double acc = ok ? S[(int64_t)i * ldS + c] : 0.0;
    const double* row = S11 + i;   // S11(i, t) at row[t * LK]
    for (int t = i + 1; t < k; ++t) acc -= row[(int64_t)t * LK] * xs[t * kSolveThreads + lane];
    const double d = row[(int64_t)i * LK];
    const double x = d != 0.0 ? acc / d : 0.0;
    xs[i * kSolveThreads + lane] = x;
    if (ok) {
      if (Z) Z[(int64_t)i * ldZ + c] = x;
      if (X) X[c * ldx + i] = static_cast<TX>(x);
    }
  }
}

// out (m x k panel) column t = A(:, J[t]): the lanes of a wave read one row of A (its k chosen entries lie
// within that row, so a wave touches one row's pages rather than one page per row), four rows per block.
template <typename T>
__global__ __launch_bounds__(256) void gather_cols_kernel(const T* __restrict__ A, int64_t lda, int64_t m,
                                                          const int* __restrict__ J, int k, T* __restrict__ out,
                                                          int64_t ldo) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= m) return;
  for (int t = threadIdx.x & 63; t < k; t += 64) out[(int64_t)t * ldo + r] = A[r * lda + J[t]];
}

// out (n x k panel, FP64) column t = A(I[t], :)^T.
template <typename T>
__global__ __launch_bounds__(256) void gather_rows_kernel(const T* __restrict__ A, int64_t lda, int64_t n,
                                                          const int* __restrict__ I, int k, double* __restrict__ out,
                                                          int64_t ldo) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y;
  if (c >= n || t >= k) return;
  out[(int64_t)t * ldo + c] = static_cast<double>(A[(int64_t)I[t] * lda + c]);
}

// v[i] = 0 where v[i] <= rel v[0] (v descending).
__global__ void cut_small_kernel(double* v, int n, double rel) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double lim = rel * v[0];
  if (v[i] <= lim) v[i] = 0.0;
}

}  // namespace

int cpqr_max_rows() { return kCpMaxL; }
int64_t cpqr_blocks(int64_t N) { return (N + kCpCols - 1) / kCpCols; }

template <typename T>
hipError_t launch_cpqr(const T* Y, int64_t ld, int64_t N, int l, int k, double* Q, int LQ, double* S, int64_t ldS,
                       double* nrm2, double* orig, double* blkmax, int* blkidx, unsigned* counter, int* J,
                       hipStream_t s) {
  if (l < 1 || l > kCpMaxL || k < 1 || k > l || N < k || LQ < l) return hipErrorInvalidValue;
  const int64_t nb = cpqr_blocks(N);
  if (nb > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  hipError_t e = launch_fill_int(reinterpret_cast<int*>(counter), 1, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((cpqr_init_kernel<T>), dim3((unsigned)nb), dim3(kCpThreads), 0, s, Y, ld, N, l, Q, LQ, S, ldS,
                     nrm2, orig, blkmax, blkidx, counter, J);
  for (int j = 0; j < k; ++j)
    hipLaunchKernelGGL((cpqr_step_kernel<T>), dim3((unsigned)nb), dim3(kCpThreads), 0, s, Y, ld, N, l, j, k, Q, LQ,
                       S, ldS, nrm2, orig, blkmax, blkidx, counter, J);
  return hipGetLastError();
}
template hipError_t launch_cpqr<float>(const float*, int64_t, int64_t, int, int, double*, int, double*, int64_t,
                                       double*, double*, double*, int*, unsigned*, int*, hipStream_t);
template hipError_t launch_cpqr<double>(const double*, int64_t, int64_t, int, int, double*, int, double*, int64_t,
                                        double*, double*, double*, int*, unsigned*, int*, hipStream_t);

template <typename TX>
hipError_t launch_id_solve(const double* S, int64_t ldS, int64_t N, int k, const int* J, double* S11, int LK,
                           double* Z, int64_t ldZ, TX* X, int64_t ldx, hipStream_t s) {
  if (k < 1 || k > kCpMaxL || LK < k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cpqr_s11_kernel, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, s, S, ldS, k, J, S11, LK);
  const size_t sh = (size_t)k * kSolveThreads * sizeof(double);
  hipLaunchKernelGGL((id_solve_kernel<TX>), dim3((unsigned)((N + kSolveThreads - 1) / kSolveThreads)),
                     dim3(kSolveThreads), sh, s, S, ldS, N, k, S11, LK, Z, ldZ, X, ldx);
  return hipGetLastError();
}
template hipError_t launch_id_solve<float>(const double*, int64_t, int64_t, int, const int*, double*, int, double*,
                                           int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_id_solve<double>(const double*, int64_t, int64_t, int, const int*, double*, int, double*,
                                            int64_t, double*, int64_t, hipStream_t);

template <typename T>
hipError_t launch_gather_cols(const T* A, int64_t lda, int64_t m, const int* J, int k, T* out, int64_t ldo,
                              hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL((gather_cols_kernel<T>), dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, A, lda, m, J, k, out,
                     ldo);
  return hipGetLastError();
}
template hipError_t launch_gather_cols<float>(const float*, int64_t, int64_t, const int*, int, float*, int64_t,
                                              hipStream_t);
template hipError_t launch_gather_cols<double>(const double*, int64_t, int64_t, const int*, int, double*, int64_t,
                                               hipStream_t);

template <typename T>
hipError_t launch_gather_rows(const T* A, int64_t lda, int64_t n, const int* I, int k, double* out, int64_t ldo,
                              hipStream_t s) {
  if (n <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL((gather_rows_kernel<T>), dim3((unsigned)((n + 255) / 256), (unsigned)k), dim3(256), 0, s, A, lda,
                     n, I, k, out, ldo);
  return hipGetLastError();
}
template hipError_t launch_gather_rows<float>(const float*, int64_t, int64_t, const int*, int, double*, int64_t,
                                              hipStream_t);
template hipError_t launch_gather_rows<double>(const double*, int64_t, int64_t, const int*, int, double*, int64_t,
                                               hipStream_t);

hipError_t launch_cut_small(double* v, int n, double rel, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cut_small_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, rel);
  return hipGetLastError();
}

}  // namespace rsvd
