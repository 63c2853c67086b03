// Multi-workgroup forms of the two small FP64 factorisations for l > 128:
// the Cholesky factorisation (with R^-1) of CholeskyQR's Gram matrix, and the
// one-sided Jacobi SVD of the l x l factor of Stage B.  Both keep the meaning
// of the one-workgroup kernels in chol.hip and jacobi.hip; only the schedule
// changes, so that the work of a step is spread over many compute units.
//
// Cholesky (right-looking, 64 x 64 blocks, working matrix M row-major LB x LB),
// with the elimination also applied to an identity block, E (= R^-T at the
// end, lower triangular, kept in the strictly lower blocks of X), as the
// one-workgroup kernel of chol.hip does:
//   for each block column J:
//     factor the diagonal block (one workgroup running the one-workgroup
//     kernel's block elimination of chol.hip on the 64 x 64 block, dependent
//     columns dropped against the original diagonal) -> R_JJ and
//     S_JJ = R_JJ^-1 (X's diagonal block; E_JJ = S_JJ^T);
//     R_JK = S_JJ^T M_JK for the blocks K > J of the block row, and
//     E_JM = S_JJ^T E_JM for the blocks M < J (one launch);
//     M_KL -= R_JK^T R_JL for J < K <= L, and E_KM -= R_JK^T E_JM for K > J,
//     M <= J (one launch).
//   R^-1(k, c) (k <= c) is then S_JJ(k, c) inside a diagonal block and E(c, k)
//   elsewhere: no separate back substitution (it was eight sequential
//   launches at l = 520).
// Dropped columns give zero rows of R and zero rows and columns of R^-1, as
// in the one-workgroup kernel.
//
// Jacobi (block one-sided, X = R^T): the columns are split into blocks of W;
// the blocks are paired by the round-robin (circle) ordering, and one
// workgroup per pair forms the Gram matrix of the pair's 2W columns, runs
// Jacobi rotations on it (the rotations the columns would take, with the
// same rotation and test as jacobi.hip) and applies the accumulated rotation
// to the columns: in the first round of a sweep, where every block sits in
// one pair, a full cyclic sweep over the 2W columns; in the other rounds only
// the pairs across the two blocks.  A sweep of nbk-1 rounds thus visits every
// pair of columns once; sweeps repeat until one passes in which no workgroup
// rotated.  All sweeps run in one persistent launch
// (workgroup g takes block pair g of every round, grid barriers between the
// rounds), which stops by itself after the converged sweep: no host
// synchronisation, and no launches spent past convergence.
#include <algorithm>

#include "internal.hpp"

namespace rsvd {

constexpr int CB = 64;   // Cholesky block

__global__ void bc_init_kernel(const double* __restrict__ g, int64_t ldg, int l, int LB, double* __restrict__ M,
                               double* __restrict__ X, double* __restrict__ gdiag, const int* __restrict__ skip) {
  if (skip && *skip) return;   // a skipped second CholeskyQR pass
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)LB * LB) return;
  const int a = (int)(t / LB), b = (int)(t - (t / LB) * LB);
  const double v = (a <= b && b < l) ? g[(int64_t)b * ldg + a] : 0.0;
  M[t] = v;
  X[t] = 0.0;   // the identity's elimination starts from zero off the diagonal blocks
  if (a == b) gdiag[a] = v;
}

// 64 x 64 tile product on the FP64 MFMA for a workgroup of four waves: wave w accumulates the output tiles
// (w, tb), tb = 0..3, of C(a, b) = sum_t A(t, a) B(t, b) over t < 64 into acc[tb] (element e of lane
// (g, j) is C(16 w + g + 4 e, 16 tb + j)); fa(t, a) and fb(t, b) load the operands (straight from memory:
// the tiles stay in L2).  sign = -1 subtracts.
template <typename FA, typename FB>
__device__ __forceinline__ void tile64(FA fa, FB fb, double sign, f64x4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int s = 0; s < CB / 4; ++s) {
    const int t = 4 * s + g;
    const double av = sign * fa(t, 16 * w + i);
    double bv[4];
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) bv[tb] = fb(t, 16 * tb + i);
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tb], acc[tb], 0, 0, 0);
  }
}

// R_JK = S_JJ^T M_JK for the blocks K = J+1+blockIdx.x (blockIdx.x < nr), and E_JM = S_JJ^T E_JM for
// M = blockIdx.x - nr < J.  In place: every product is complete before the workgroup barrier, the stores
// come after it.
__global__ __launch_bounds__(256) void bc_panel_kernel(double* __restrict__ M, double* __restrict__ X, int LB, int j0,
                                                       int nr, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const bool erow = (int)blockIdx.x >= nr;
  double* blk = erow ? X + (int64_t)j0 * LB + CB * ((int)blockIdx.x - nr) : M + (int64_t)j0 * LB + j0 + CB * (1 + blockIdx.x);
  const double* S = X + (int64_t)j0 * LB + j0;
  f64x4 acc[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) acc[tb] = f64x4{0.0, 0.0, 0.0, 0.0};
  tile64([&](int t, int a) { return S[(int64_t)t * LB + a]; }, [&](int t, int b) { return blk[(int64_t)t * LB + b]; },
         1.0, acc);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int e = 0; e < 4; ++e) blk[(int64_t)(16 * w + g + 4 * e) * LB + 16 * tb + i] = acc[tb][e];
}

// M_KL -= R_JK^T R_JL for J < K <= L (the first nr (nr + 1) / 2 workgroups enumerate the pairs (K, L)), and
// E_KM -= R_JK^T E_JM for K > J, M <= J (the rest, nr (J + 1) of them; E_JJ = S_JJ^T).  The output block
// is never an operand.
__global__ __launch_bounds__(256) void bc_trail_kernel(double* __restrict__ M, double* __restrict__ X, int LB, int j0,
                                                       int nr, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int jb = j0 / CB;
  const int npair = nr * (nr + 1) / 2;
  const double* A;
  const double* B;
  int64_t sbt = LB, sbb = 1;
  double* out;
  if ((int)blockIdx.x < npair) {
    int idx = blockIdx.x, kb = 0;
    while (idx >= nr - kb) { idx -= nr - kb; ++kb; }
    const int lb = kb + idx;
    const int k0 = j0 + CB * (1 + kb), l0 = j0 + CB * (1 + lb);
    A = M + (int64_t)j0 * LB + k0;
    B = M + (int64_t)j0 * LB + l0;
    out = M + (int64_t)k0 * LB + l0;
  } else {
    const int idx = (int)blockIdx.x - npair;
    const int kb = idx / (jb + 1), mb = idx - (idx / (jb + 1)) * (jb + 1);
    const int k0 = j0 + CB * (1 + kb), m0 = CB * mb;
    A = M + (int64_t)j0 * LB + k0;
    if (mb < jb) {
      B = X + (int64_t)j0 * LB + m0;
    } else {   // E_JJ(t, b) = S_JJ(b, t)
      B = X + (int64_t)j0 * LB + j0;
      sbt = 1;
      sbb = LB;
    }
    out = X + (int64_t)k0 * LB + m0;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, i = lane & 15;
  f64x4 acc[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[tb][e] = out[(int64_t)(16 * w + g + 4 * e) * LB + 16 * tb + i];
  tile64([&](int t, int a) { return A[(int64_t)t * LB + a]; }, [&](int t, int b) { return B[t * sbt + b * sbb]; },
         -1.0, acc);
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(int64_t)(16 * w + g + 4 * e) * LB + 16 * tb + i] = acc[tb][e];
}

// rinv_p[c*LP + k] = R^-1(k, c) for c, k < l; the identity on the padding (everywhere for a skipped pass).
template <typename TQ>
__global__ void bc_rinv_out_kernel(const double* __restrict__ X, int LB, int l, int LP, TQ* __restrict__ rinv_p,
                                   const int* __restrict__ skip) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)LP * LP) return;
  const int c = (int)(t / LP), k = (int)(t - (t / LP) * LP);
  double v;
  if (c >= l || k >= l || (skip && *skip)) v = (c == k) ? 1.0 : 0.0;
  else if (k > c) v = 0.0;
  else v = (k / CB == c / CB) ? X[(int64_t)k * LB + c] : X[(int64_t)c * LB + k];   // S_JJ, or E(c, k)
  rinv_p[t] = static_cast<TQ>(v);
}

// r_out (row-major LP x LP) = R, or R R_prev when r_prev is given; identity on the padding.
// One 64 x 64 tile (I <= J) per workgroup.
__global__ __launch_bounds__(256) void bc_r_out_kernel(const double* __restrict__ M, int LB, int l, int LP,
                                                       const double* __restrict__ r_prev, double* __restrict__ r_out,
                                                       int nbk) {
  const int tid = threadIdx.x;
  int idx = blockIdx.x, ib = 0;
  while (idx >= nbk - ib) { idx -= nbk - ib; ++ib; }
  const int jb = ib + idx;
  const int i0 = ib * CB, j0 = jb * CB;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, li = lane & 15;
  f64x4 acc[4];
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) acc[tb] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (r_prev) {
    // sum over K = I .. J of M_IK R_prev_KJ: A(t, a) = M(i0 + a, k0 + t), B(t, b) = R_prev(k0 + t, j0 + b)
    for (int kb = ib; kb <= jb; ++kb) {
      const int k0 = kb * CB;
      tile64([&](int t, int a) { return M[(int64_t)(i0 + a) * LB + k0 + t]; },
             [&](int t, int b) {
               const int kk = k0 + t, jj = j0 + b;
               return (kk < l && jj < l) ? r_prev[(int64_t)kk * LP + jj] : 0.0;
             },
             1.0, acc);
    }
  } else {
#pragma unroll
    for (int tb = 0; tb < 4; ++tb)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[tb][e] = M[(int64_t)(i0 + 16 * w + g + 4 * e) * LB + j0 + 16 * tb + li];
  }
#pragma unroll
  for (int tb = 0; tb < 4; ++tb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = i0 + 16 * w + g + 4 * e, b = j0 + 16 * tb + li;
      if (a >= LP || b >= LP) continue;
      double v;
      if (a >= l || b >= l) v = (a == b) ? 1.0 : 0.0;
      else v = (b >= a) ? acc[tb][e] : 0.0;
      r_out[(int64_t)a * LP + b] = v;
    }
  // the strictly lower tiles (I > J) are zero
  if (ib != jb) {
    for (int t = tid; t < CB * CB; t += 256) {
      const int r = t / CB, c = t - (t / CB) * CB;
      const int a = j0 + r, b = i0 + c;   // tile (J, I), below the diagonal
      if (a < LP && b < LP) r_out[(int64_t)a * LP + b] = (a >= l || b >= l) ? (a == b ? 1.0 : 0.0) : 0.0;
    }
  }
}

size_t chol_blocked_scratch_doubles(int LP) {
  const size_t LB = (size_t)(LP + CB - 1) / CB * CB;
  return 2 * LB * LB + LB;
}

// The skip test of the blocked form (as the one-workgroup Cholesky kernel's): *skip_out = 1 when
// l sum_i G_ii ||row i of R^-1||^2 <= kappa_max^2, never when a pivot was dropped (a zero on the diagonal of
// R^-1) or a value is not finite.  Each stored entry of X is one entry of R^-1: X(a, b) with a <= b inside a
// diagonal block is R^-1(a, b) (weight G_aa); X(a, b) below the diagonal blocks is R^-1(b, a) (weight G_bb).
// So row a of X, read contiguously by one wave, gives part[a]; a zero pivot makes part[a] NaN.
__global__ __launch_bounds__(256) void bc_bound_part_kernel(const double* __restrict__ X, int LB, int l,
                                                            const double* __restrict__ gdiag,
                                                            double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= l) return;
  const double* xa = X + (int64_t)a * LB;
  const int d0 = a / CB * CB;
  const int bend = min(d0 + CB, l);
  const double ga = gdiag[a];
  double f = 0.0;
  for (int b = lane; b < bend; b += 64) {
    if (b >= d0 && b < a) continue;   // the unused lower triangle of the diagonal block
    const double v = xa[b];
    f = fma(b >= d0 ? ga : gdiag[b], v * v, f);
  }
  f = wave_sum(f);
  if (lane == 0) part[a] = xa[a] != 0.0 ? f : __longlong_as_double(0x7ff8000000000000LL);
}

__global__ __launch_bounds__(1024) void bc_bound_fin_kernel(const double* __restrict__ part, int l,
                                                            double kappa2_max, int* __restrict__ skip_out) {
  __shared__ double w[16];
  double f = threadIdx.x < l ? part[threadIdx.x] : 0.0;
  f = wave_sum(f);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += w[i];
    *skip_out = ((double)l * t <= kappa2_max) ? 1 : 0;   // false for NaN
  }
}

template <typename TQ>
hipError_t launch_chol_blocked(const double* g, int64_t ldg, int l, int LP, double tau, TQ* rinv_p, double* r_out,
                               const double* r_prev, double* scratch, int* flags, hipStream_t s, int* skip_out,
                               double kappa2_max, const int* skip_in) {
  const int LB = (LP + CB - 1) / CB * CB;
  const int nbk = LB / CB;
  double* M = scratch;
  double* X = M + (size_t)LB * LB;
  double* gdiag = X + (size_t)LB * LB;
  const int64_t ll = (int64_t)LB * LB;
  hipLaunchKernelGGL(bc_init_kernel, dim3((unsigned)((ll + 255) / 256)), dim3(256), 0, s, g, ldg, l, LB, M, X,
                     gdiag, skip_in);
  // X: S_JJ on the diagonal blocks, E below them; its blocks above the diagonal are never read.  With skip_in
  // set on the device every launch returns at once and R^-1 comes out as the identity.
  for (int jb = 0; jb < nbk; ++jb) {
    const int j0 = jb * CB;
    hipError_t e = launch_chol_diag64(M, LB, j0, l, gdiag, tau, X, flags, s, skip_in);
    if (e != hipSuccess) return e;
    const int nr = nbk - 1 - jb;
    if (nr + jb > 0)
      hipLaunchKernelGGL(bc_panel_kernel, dim3((unsigned)(nr + jb)), dim3(256), 0, s, M, X, LB, j0, nr, skip_in);
    if (nr > 0)
      hipLaunchKernelGGL(bc_trail_kernel, dim3((unsigned)(nr * (nr + 1) / 2 + nr * (jb + 1))), dim3(256), 0, s, M, X,
                         LB, j0, nr, skip_in);
  }
  const int64_t lp2 = (int64_t)LP * LP;
  hipLaunchKernelGGL((bc_rinv_out_kernel<TQ>), dim3((unsigned)((lp2 + 255) / 256)), dim3(256), 0, s, X, LB, l, LP,
                     rinv_p, skip_in);
  if (r_out)
    hipLaunchKernelGGL(bc_r_out_kernel, dim3((unsigned)(nbk * (nbk + 1) / 2)), dim3(256), 0, s, M, LB, l, LP, r_prev,
                       r_out, nbk);
  if (skip_out) {   // M is free once R is out: it holds the per-row partials
    hipLaunchKernelGGL(bc_bound_part_kernel, dim3((unsigned)((l + 3) / 4)), dim3(256), 0, s, X, LB, l, gdiag, M);
    hipLaunchKernelGGL(bc_bound_fin_kernel, dim3(1), dim3(1024), 0, s, M, l, kappa2_max, skip_out);
  }
  return hipGetLastError();
}

template hipError_t launch_chol_blocked<float>(const double*, int64_t, int, int, double, float*, double*,
                                               const double*, double*, int*, hipStream_t, int*, double, const int*);
template hipError_t launch_chol_blocked<double>(const double*, int64_t, int, int, double, double*, double*,
                                                const double*, double*, int*, hipStream_t, int*, double,
                                                const int*);

// ---------------------------------------------------------------------------
// Block one-sided Jacobi
// ---------------------------------------------------------------------------

__device__ __forceinline__ int bj_player(int pos, int round, int le) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (le - 1);
}

// xs: column p of X at xs[p*ldx + i], i < LP (rows l .. LP-1 and columns past l are zero).
__global__ void bj_init_kernel(const double* __restrict__ R, int l, int LP, double* __restrict__ xs, int ldx,
                               int ncols) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)ncols * ldx) return;
  const int p = (int)(t / ldx), i = (int)(t - (t / ldx) * ldx);
  xs[t] = (p < l && i < l) ? R[(int64_t)p * LP + i] : 0.0;
}

// 1/x and 1/sqrt(x) for finite x > 0: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double bj_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double bj_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// Control words: the per-sweep rotation counts (sweeps < kBlockedSweepCap), then the deflation bound
// (a double in words 60-61), the barrier's arrival count and the time-out flag.
constexpr int kBjCtlWords = 64;
constexpr int kBjCtlThr2 = 60;      // tol^2 ||X||_F^2, as a double
constexpr int kBjCtlBarrier = 62;   // arrivals at the grid barrier, cumulative
constexpr int kBjCtlTimeout = 63;   // set when a barrier wait ran out of time
constexpr int kBlockedSweepCap = 60;

// *thr2 = tol^2 ||X||_F^2 (one workgroup of 1024 threads, partial sums in a fixed order): a column whose
// squared norm is at or below it is numerically zero (no rotation; sigma = 0 and a zero vector).
__global__ __launch_bounds__(1024) void bj_fro_kernel(const double* __restrict__ xs, int ldx, int l, double tol,
                                                      double* __restrict__ thr2) {
  __shared__ double part[16];
  // rows l .. ldx-1 of the first l columns are zero, so the l ldx values are summed as one flat range
  const int64_t n = (int64_t)l * ldx;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0;
  int64_t t = threadIdx.x;
  for (; t + 3 * 1024 < n; t += 4 * 1024) {
    const double a = xs[t], b = xs[t + 1024], c = xs[t + 2048], d = xs[t + 3072];
    f0 = fma(a, a, f0);
    f1 = fma(b, b, f1);
    f2 = fma(c, c, f2);
    f3 = fma(d, d, f3);
  }
  for (; t < n; t += 1024) f0 = fma(xs[t], xs[t], f0);
  double f = (f0 + f1) + (f2 + f3);
  f = wave_sum(f);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += part[w];
    *thr2 = tol * tol * t;
  }
}

// Grid-wide barrier between the rounds of the persistent kernel.  Every workgroup of the grid is resident
// (the host checks the occupancy before the launch), so the wait ends; it is still bounded by tick_limit
// ticks of the constant wall clock, after which the caller gives up.  The stores of every thread are made
// visible at agent scope before the arrival (the L2 caches of the compute dies are not coherent for plain
// stores), and every thread acquires at agent scope after the wait.  Returns false (uniformly within the
// workgroup) on time-out.
__device__ __forceinline__ bool bj_grid_barrier(int* count, int target, long long tick_limit, int* ok_sh) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(count, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = (long long)wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if ((long long)wall_clock64() - t0 > tick_limit) {
        ok = 0;
        break;
      }
    }
    *ok_sh = ok;
  }
  __syncthreads();
  __threadfence();
  return *ok_sh != 0;
}

template <int W>
struct BjShared {
  double rc[W], rs[W], rt[W];   // the inner round's rotations, one per disjoint pair
  int any_rot;
  int need;   // a pair of the inner sweep passes the rotation test on G as assembled
  int ok;
};

// One pair step of the block one-sided Jacobi on the NC = 2W columns of block pair `pair` of round `round`:
//   1. G = X^T X of the pair's columns on the FP64 MFMA (each wave a share of the 16-row slabs, the wave
//      partials summed in a fixed order through LDS);
//   2. inner rounds of NC/2 disjoint rotations on G in LDS (a full cyclic sweep in round 0 of a sweep, the
//      cross-block pairs in the others; below): each rotation is the one the columns themselves would take
//      (G's entries are their inner products; the same test and rotation as the one-workgroup kernel),
//      computed once per pair and inner round, G is carried along as J^T G J (2 x 2 blocks, the pair's own
//      block updated exactly), and V = J_1 J_2 ... is accumulated;
//   3. X <- X V on the FP64 MFMA, slab by slab in place, if anything rotated (counted in *rot).
template <int W>
__device__ __forceinline__ void bj_pair_step(double* __restrict__ xs, int ldx, int LP, int nbk, int pair, int round,
                                             double tol, double thr2, int* __restrict__ rot, double* lds,
                                             BjShared<W>& sh) {
  // Inner rounds: in round 0 of a sweep (every block in exactly one pair) a full cyclic sweep over the
  // 2W columns, NC - 1 rounds in circle order, which also meets every pair inside a block; in the other
  // rounds only the W x W cross pairs, W rounds of W disjoint pairs (p = k, q = W + (k + ir) mod W).  Each
  // column pair is thus visited once per sweep.
  const bool full = round == 0;
  constexpr int NC = 2 * W;                 // columns of the block pair
  constexpr int NT = NC / 16;               // 16-column MFMA tiles (1 or 2)
  constexpr int NTT = NT * (NT + 1) / 2;    // tiles on and above the diagonal of G
  constexpr int NP = NC / 2;                // disjoint inner pairs per round
  double* red = lds;                        // [8 waves][NTT tiles][256]
  double* gb = red + 8 * NTT * 256;         // two NC x NC buffers of G (row-major)
  double* vm = gb + 2 * NC * NC;            // V, NC x NC row-major
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ci = lane & 15, g = lane >> 4;
  const int bI = bj_player(pair, round, nbk), bJ = bj_player(nbk - 1 - pair, round, nbk);
  auto gcol = [&](int c) { return c < W ? bI * W + c : bJ * W + (c - W); };
  const int nslab = LP / 16;

  // 1. Gram.  Lane (ci, g) of slab sl loads rows 16 sl + 4 g + e (e = 0..3) of pair column 16 t + ci; MFMA
  // step e takes contraction index g <-> row 16 sl + 4 g + e for both operands.
  {
    const double* colp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) colp[t] = xs + (int64_t)gcol(16 * t + ci) * ldx + 4 * g;
    f64x4 acc[NTT];
#pragma unroll
    for (int t = 0; t < NTT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    // SB slabs of a wave are loaded before their MFMAs (32 values in flight per lane), so a round pays one
    // memory latency per batch rather than one per slab.
    constexpr int SB = NT == 2 ? 4 : 8;
    for (int s0 = wave; s0 < nslab; s0 += 8 * SB) {
      double x[SB][NT][4];
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        const int sl = s0 + 8 * b;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (sl < nslab) {
            const double2 u = *reinterpret_cast<const double2*>(colp[t] + 16 * sl);
            const double2 v = *reinterpret_cast<const double2*>(colp[t] + 16 * sl + 2);
            x[b][t][0] = u.x; x[b][t][1] = u.y; x[b][t][2] = v.x; x[b][t][3] = v.y;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        if (s0 + 8 * b >= nslab) break;   // uniform in the wave
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[b][0][e], x[b][0][e], acc[0], 0, 0, 0);
          if constexpr (NT == 2) {
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[b][0][e], x[b][1][e], acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[b][1][e], x[b][1][e], acc[2], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NTT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(wave * NTT + t) * 256 + r * 64 + lane] = acc[t][r];
  }
  if (tid == 0) {
    sh.any_rot = 0;
    sh.need = 0;
  }
  for (int e = tid; e < NC * NC; e += 512) vm[e] = (e / NC == e % NC) ? 1.0 : 0.0;
  __syncthreads();
  // Wave partials summed in wave order.  Accumulator element r of lane L holds G(L/16 + 4 r, L % 16) of its
  // tile; tile index 0 = (0,0), 1 = (0,1), 2 = (1,1).  The entries on and above the diagonal are kept and
  // mirrored, so G is exactly symmetric.
  for (int e = tid; e < NTT * 256; e += 512) {
    const int t = e >> 8, idx = e & 255, r = idx >> 6, L = idx & 63;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < 8; ++w) v += red[(w * NTT + t) * 256 + idx];
    const int ta = (t == 2) ? 1 : 0, tb = (t == 0) ? 0 : 1;
    const int a = 16 * ta + (L >> 4) + 4 * r, b = 16 * tb + (L & 15);
    if (ta != tb || a <= b) {
      gb[a * NC + b] = v;
      gb[b * NC + a] = v;
    }
  }
  __syncthreads();

  // 2. One inner sweep on G.
  auto pq = [&](int k, int ir, int& p, int& q) {
    if (full) {
      p = bj_player(k, ir, NC);
      q = bj_player(NC - 1 - k, ir, NC);
    } else {
      p = k;
      q = W + ((k + ir) & (W - 1));
    }
  };
  // G changes only by rotations, so when no pair the inner sweep visits (every pair in a full sweep, the
  // cross pairs otherwise) passes the rotation test on G as assembled, no inner round rotates: the sweep is
  // skipped, with exactly the result of running it.
  for (int e = tid; e < NC * NC; e += 512) {
    const int p = e / NC, q = e - (e / NC) * NC;
    if (p < q && (full || (p < W && q >= W))) {
      const double al = gb[p * NC + p], be = gb[q * NC + q], ga = gb[p * NC + q];
      if (al > thr2 && be > thr2 && fabs(ga) > tol * (sqrt(al) * sqrt(be))) sh.need = 1;
    }
  }
  __syncthreads();
  const int nir = sh.need == 0 ? 0 : full ? NC - 1 : W;
  int cur = 0;
  for (int ir = 0; ir < nir; ++ir) {
    const double* G = gb + cur * NC * NC;
    double* Gn = gb + (cur ^ 1) * NC * NC;
    // a. the rotation of each disjoint pair of this inner round: rotate when |g_pq| > tol sqrt(g_pp) sqrt(g_qq)
    // and neither column is numerically zero (g_pp, g_qq > thr2);
    // t = tan of the angle that zeroes g_pq (the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (g_qq - g_pp) /
    // (2 g_pq)), x_p' = c x_p - s x_q, x_q' = s x_p + c x_q.  t == 0 (an angle below the double range) means
    // no rotation everywhere below.
    if (tid < NP) {
      int p, q;
      pq(tid, ir, p, q);
      const double al = G[p * NC + p], be = G[q * NC + q], ga = G[p * NC + q];
      double c = 1.0, s = 0.0, t = 0.0;
      if (al > thr2 && be > thr2 && fabs(ga) > tol * (sqrt(al) * sqrt(be))) {
        const double zeta = (be - al) * bj_rcp(2.0 * ga);
        if (fabs(zeta) > 1e150) {
          t = 0.5 * bj_rcp(zeta);
        } else {
          const double z2 = 1.0 + zeta * zeta;
          t = bj_rcp(fabs(zeta) + z2 * bj_rsq(z2));
          t = zeta >= 0.0 ? t : -t;
        }
        c = bj_rsq(1.0 + t * t);
        s = c * t;
        if (t != 0.0) sh.any_rot = 1;
      }
      sh.rc[tid] = c;
      sh.rs[tid] = s;
      sh.rt[tid] = t;
    }
    __syncthreads();
    // b. G <- J^T G J by 2 x 2 blocks (block (kr, kc) = rows of pair kr, columns of pair kc), V <- V J.
    if (tid < NP * NP) {
      const int kr = tid / NP, kc = tid - (tid / NP) * NP;
      int pr, qr, pc, qc;
      pq(kr, ir, pr, qr);
      pq(kc, ir, pc, qc);
      if (kr == kc) {
        const double ar = G[pr * NC + pr], br = G[qr * NC + qr], gr = G[pr * NC + qr];
        const double tr = sh.rt[kr];
        const bool rr = tr != 0.0;
        Gn[pr * NC + pr] = rr ? ar - tr * gr : ar;
        Gn[qr * NC + qr] = rr ? br + tr * gr : br;
        Gn[pr * NC + qr] = rr ? 0.0 : gr;
        Gn[qr * NC + pr] = rr ? 0.0 : gr;
      } else {
        const double cr = sh.rc[kr], sr = sh.rs[kr], cc = sh.rc[kc], sc = sh.rs[kc];
        const double b00 = G[pr * NC + pc], b01 = G[pr * NC + qc], b10 = G[qr * NC + pc], b11 = G[qr * NC + qc];
        // B J_c, then J_r^T (B J_c)
        const double t00 = b00 * cc - b01 * sc, t01 = b00 * sc + b01 * cc;
        const double t10 = b10 * cc - b11 * sc, t11 = b10 * sc + b11 * cc;
        Gn[pr * NC + pc] = cr * t00 - sr * t10;
        Gn[pr * NC + qc] = cr * t01 - sr * t11;
        Gn[qr * NC + pc] = sr * t00 + cr * t10;
        Gn[qr * NC + qc] = sr * t01 + cr * t11;
      }
    } else if (tid >= 256) {
      for (int item = tid - 256; item < NC * NP; item += 256) {
        const int i = item / NP, k = item - (item / NP) * NP;
        if (sh.rt[k] != 0.0) {
          int p, q;
          pq(k, ir, p, q);
          const double c = sh.rc[k], sn = sh.rs[k];
          const double vp = vm[i * NC + p], vq = vm[i * NC + q];
          vm[i * NC + p] = c * vp - sn * vq;
          vm[i * NC + q] = sn * vp + c * vq;
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  const bool rotated = sh.any_rot != 0;

  // 3. X <- X V: output tile jt of slab sl is D(j, i) = sum_k V(k, 16 jt + j) X(16 sl + i, k), with the A
  // operand V^T read from LDS and the B operand X^T (16 lanes read 16 consecutive rows of one column).
  if (rotated) {
    double vf[NT][NC / 4];   // this lane's V^T operands, the same for every slab
#pragma unroll
    for (int jt = 0; jt < NT; ++jt)
#pragma unroll
      for (int st = 0; st < NC / 4; ++st) vf[jt][st] = vm[(4 * st + g) * NC + 16 * jt + ci];
    constexpr int SX = NT == 2 ? 4 : 8;   // slabs loaded ahead per batch (32 values per lane)
    for (int s0 = wave; s0 < nslab; s0 += 8 * SX) {
      double xv[SX][NC / 4];
#pragma unroll
      for (int b = 0; b < SX; ++b) {
        const int sl = s0 + 8 * b;
        if (sl < nslab) {
#pragma unroll
          for (int st = 0; st < NC / 4; ++st) xv[b][st] = xs[(int64_t)gcol(4 * st + g) * ldx + 16 * sl + ci];
        }
      }
#pragma unroll
      for (int b = 0; b < SX; ++b) {
        const int sl = s0 + 8 * b;
        if (sl >= nslab) break;   // uniform in the wave
        const int i = 16 * sl + ci;
#pragma unroll
        for (int jt = 0; jt < NT; ++jt) {
          f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int st = 0; st < NC / 4; ++st)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vf[jt][st], xv[b][st], acc, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) xs[(int64_t)gcol(16 * jt + g + 4 * r) * ldx + i] = acc[r];
        }
      }
    }
    if (tid == 0) atomicAdd(rot, 1);
  }
}

// All sweeps in one launch: workgroup g takes block pair g of every round, a grid barrier separates the
// rounds, and the loop ends after the first sweep in which no workgroup rotated (every workgroup reads the
// same count after that sweep's last barrier) or after cap sweeps.  ctl[s] counts the pair steps of sweep s
// that rotated.
template <int W>
__global__ __launch_bounds__(512) void bj_sweeps_kernel(double* __restrict__ xs, int ldx, int LP, int nbk,
                                                        double tol, int cap, int* __restrict__ ctl,
                                                        long long tick_limit) {
  extern __shared__ double lds[];
  __shared__ BjShared<W> sh;
  const double thr2 = *reinterpret_cast<const double*>(ctl + kBjCtlThr2);
  int arrivals = 0;
  for (int sweep = 0; sweep < cap; ++sweep) {
    for (int round = 0; round < nbk - 1; ++round) {
      bj_pair_step<W>(xs, ldx, LP, nbk, blockIdx.x, round, tol, thr2, ctl + sweep, lds, sh);
      arrivals += gridDim.x;
      if (!bj_grid_barrier(ctl + kBjCtlBarrier, arrivals, tick_limit, &sh.ok)) {
        if (threadIdx.x == 0) __hip_atomic_store(ctl + kBjCtlTimeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    if (__hip_atomic_load(ctl + sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
  }
}

// flags[3] = sweeps run (the first with no rotation included), flags[2] += 1 if every sweep run rotated; a
// barrier time-out counts in flags[0] and flags[2].
__global__ void bj_flags_kernel(int* flags, const int* ctl, int cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int s = 0;
    while (s < cap && ctl[s] != 0) ++s;
    const bool timeout = ctl[kBjCtlTimeout] != 0;
    if (s == cap || timeout) atomicAdd(&flags[2], 1);
    if (timeout) atomicAdd(&flags[0], 1);
    atomicMax(&flags[3], s < cap ? s + 1 : cap);
  }
}

size_t jacobi_blocked_scratch_bytes(int LP) {
  return (size_t)(LP + 32) * LP * sizeof(double) + kBjCtlWords * sizeof(int);
}

template <typename TU>
hipError_t jacobi_epilogue_launch(const double* xs, int ldx, int l, int LP, const double* thr2, double* sigma,
                                  double* uhat_d, TU* uhat_p, TU* vhat_p, hipStream_t s);

template <int W>
constexpr size_t bj_lds_bytes() {
  return (size_t)(8 * ((2 * W / 16) * (2 * W / 16 + 1) / 2) * 256 + 3 * (2 * W) * (2 * W)) * sizeof(double);
}

// Sets the kernel's LDS limit once and checks that `grid` workgroups of it fit on the device at once (the
// barrier needs every workgroup resident).
template <int W>
hipError_t bj_prepare(int grid) {
  static int resident = -1;   // workgroups the device holds at once, -1 until known
  if (resident < 0) {
    const void* f = reinterpret_cast<const void*>(&bj_sweeps_kernel<W>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bj_lds_bytes<W>());
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 512, bj_lds_bytes<W>())) != hipSuccess)
      return e;
    resident = cus * per_cu;
  }
  return grid <= resident ? hipSuccess : hipErrorCooperativeLaunchTooLarge;
}

template <typename TU>
hipError_t launch_jacobi_blocked(const double* R, int l, int LP, double tol, int max_sweeps, double* sigma,
                                 double* uhat_d, TU* uhat_p, TU* vhat_p, double* scratch, int* flags, hipStream_t s) {
  // W = 16 (32-column pair steps) up to l = 600, W = 8 beyond (the block count stays within the circle
  // method's range and the columns past l within the scratch).
  const int W = l <= 600 ? 16 : 8;
  int nbk = (l + W - 1) / W;
  nbk += nbk & 1;
  const int ldx = LP;
  double* xs = scratch;
  int* ctl = reinterpret_cast<int*>(scratch + (size_t)(LP + 32) * LP);
  const int ncols = nbk * W;
  if (ncols > LP + 32 || LP % 16 != 0) return hipErrorInvalidValue;
  const int grid = nbk / 2;
  hipError_t e = W == 16 ? bj_prepare<16>(grid) : bj_prepare<8>(grid);
  if (e != hipSuccess) return e;
  int dev = 0, khz = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return e;
  const long long tick_limit = (long long)std::max(khz, 1000) * 2000;   // two seconds per barrier wait
  const int64_t tot = (int64_t)ncols * ldx;
  hipLaunchKernelGGL(bj_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R, l, LP, xs, ldx, ncols);
  if ((e = launch_fill_int(ctl, kBjCtlWords, 0, s)) != hipSuccess) return e;
  double* thr2 = reinterpret_cast<double*>(ctl + kBjCtlThr2);
  hipLaunchKernelGGL(bj_fro_kernel, dim3(1), dim3(1024), 0, s, xs, ldx, l, tol, thr2);
  const int cap = std::min(std::max(max_sweeps, 1), kBlockedSweepCap);
  if (W == 16)
    hipLaunchKernelGGL((bj_sweeps_kernel<16>), dim3((unsigned)grid), dim3(512), bj_lds_bytes<16>(), s, xs, ldx, LP,
                       nbk, tol, cap, ctl, tick_limit);
  else
    hipLaunchKernelGGL((bj_sweeps_kernel<8>), dim3((unsigned)grid), dim3(512), bj_lds_bytes<8>(), s, xs, ldx, LP,
                       nbk, tol, cap, ctl, tick_limit);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bj_flags_kernel, dim3(1), dim3(64), 0, s, flags, ctl, cap);
  return jacobi_epilogue_launch<TU>(xs, ldx, l, LP, thr2, sigma, uhat_d, uhat_p, vhat_p, s);
}

template hipError_t launch_jacobi_blocked<float>(const double*, int, int, double, int, double*, double*, float*,
                                                 float*, double*, int*, hipStream_t);
template hipError_t launch_jacobi_blocked<double>(const double*, int, int, double, int, double*, double*, double*,
                                                  double*, double*, int*, hipStream_t);

}  // namespace rsvd
