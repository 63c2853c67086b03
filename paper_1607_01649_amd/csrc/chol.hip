// Cholesky factorisation of the l x l Gram matrix of CholeskyQR, in FP64, in
// one workgroup.
//
// orth(Y) (Section 2.3: any unpivoted orthonormalisation will do) is computed
// as CholeskyQR: G = Y^T Y = R^T R, Q = Y R^-1.  This kernel factors G and at
// the same time builds R^-T by applying every elimination step to an identity
// block, so the triangular apply that follows is a plain panel product with
// R^-1 and no sequential back-substitution is needed.
//
// Elimination is run in the unscaled (L D L^T) form: at step j every row
// a > j is updated from the still-unscaled row j,
//     U(a, b) -= U(j, a) U(j, b) / d_j          (b >= a, the trailing block)
//     T(a, b) -= U(j, a) T(j, b) / d_j          (b <= j, the identity block)
// with d_j = U(j, j), so step j reads row j and writes only rows below it:
// one barrier per step.  At the end R = D^-1/2 U and R^-T = D^-1/2 T.
//
// Storage: register blocks, l <= 128; larger l goes to the blocked
// multi-workgroup form in blocked.hip.
//
// Numerically dependent columns (pivot <= tau_rel * G_jj) are dropped: they
// take no part in later eliminations, row j of R and column j of R^-1 come out
// zero (so column j of Q is exactly zero).  Counted in flags[1]; a non-finite
// pivot is counted in flags[0].
#include "internal.hpp"

namespace rsvd {

constexpr int kCholThreads = 1024;

// l <= 128: thread t owns the 4 x 4 register blocks U[4][4] and T[4][4] of
// rows a0..a0+3 and columns b0..b0+3.  A wave covers a 32 x 32 tile (wave w:
// row band w / 4, column band w % 4), so that at step j whole waves can skip:
// a wave whose rows are all <= j has nothing to do, a wave whose columns are
// all > j only updates U and one whose columns are all <= j only T.  U starts
// as G's upper triangle, T as the identity.  Step j:
//     U(a, b) -= f_a U(j, b)   for a > j, b > j      (f_a = U(j, a) / d_j)
//     T(a, b) -= f_a T(j, b)   for a > j (T(j, b) = 0 for b > j)
// with masked vectors (f zero for a <= j, U(j, b) zero for b <= j).  The
// owners of row j+1 publish U(j+1, :) and T(j+1, :) to LDS before the step's
// barrier (double-buffered), and the owner of the diagonal entry decides the
// pivot (drop test, 1/d, 1/sqrt(d)) once for everyone.
template <typename TQ>
__global__ __launch_bounds__(kCholThreads) void chol_reg_kernel(const double* __restrict__ g, int64_t ldg, int l,
                                                                 int LP, double tau_rel, TQ* __restrict__ rinv_p,
                                                                 double* __restrict__ r_out,
                                                                 const double* __restrict__ r_prev,
                                                                 int* __restrict__ flags) {
  __shared__ double urow[2][128];
  __shared__ double trow[2][128];
  __shared__ double pinv[2];      // 1/d_j of the published row, 0 for a dropped pivot
  __shared__ double gdiag[128];
  __shared__ double rsd[128];     // 1/sqrt(d_j), 0 for a dropped column
  extern __shared__ double Ufull[];   // LP x LP, filled at the end when r_out is wanted
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  const int a0 = 32 * (wv >> 2) + 4 * (ln >> 3), b0 = 32 * (wv & 3) + 4 * (ln & 7);
  const int rlast = 32 * (wv >> 2) + 31, cfirst = 32 * (wv & 3), clast = cfirst + 31;
  double U[4][4], T[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int a = a0 + i, b = b0 + k;
      U[i][k] = (a < l && b < l && a <= b) ? g[(int64_t)b * ldg + a] : 0.0;
      T[i][k] = (a == b) ? 1.0 : 0.0;
      if (a == b && a < l) gdiag[a] = U[i][k];
    }
  int bad = 0, dropped = 0;
  // pivot decision for row r (r < l) from its current diagonal d, by the diagonal's owner
  auto decide = [&](int r, double d, int buf) {
    const double gd = gdiag[r];
    const bool nonfinite = !isfinite(d) || !isfinite(gd);
    const bool drop = nonfinite || !(d > tau_rel * gd) || !(d > 0.0);
    bad += nonfinite;
    dropped += (drop && !nonfinite);
    pinv[buf] = drop ? 0.0 : 1.0 / d;
    rsd[r] = drop ? 0.0 : 1.0 / sqrt(d);
  };
  __syncthreads();   // gdiag
  if (a0 == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) { urow[0][b0 + k] = U[0][k]; trow[0][b0 + k] = T[0][k]; }
    if (b0 == 0) decide(0, U[0][0], 0);
  }
  __syncthreads();

  for (int j = 0; j < l; ++j) {
    const int buf = j & 1;
    const double dinv = pinv[buf];
    if (rlast > j && dinv != 0.0) {   // uniform over the wave
      const double* uj = urow[buf];
      const double* tj = trow[buf];
      double f[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) f[i] = (a0 + i > j) ? uj[a0 + i] * dinv : 0.0;
      if (clast > j) {
        double ub[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) ub[k] = (b0 + k > j) ? uj[b0 + k] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) U[i][k] -= f[i] * ub[k];
      }
      if (cfirst <= j) {
        double tb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) tb[k] = tj[b0 + k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) T[i][k] -= f[i] * tb[k];
      }
    }
    // (static row index: a runtime index into U/T would move them to scratch)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (a0 + i == j + 1 && j + 1 < l) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          urow[buf ^ 1][b0 + k] = U[i][k];
          trow[buf ^ 1][b0 + k] = T[i][k];
          if (b0 + k == j + 1) decide(j + 1, U[i][k], buf ^ 1);
        }
      }
    __syncthreads();
  }
  if (bad) atomicAdd(&flags[0], bad);
  if (dropped) atomicAdd(&flags[1], dropped);
  // R^-1 in panel layout: rinv_p[c*LP + k] = R^-T(c, k) = T(c, k) / sqrt(d_c); identity on padding.
  if (a0 < LP && b0 < LP) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        int c = a0 + i, kk = b0 + k;
        double v;
        if (c >= l || kk >= l) v = (c == kk) ? 1.0 : 0.0;
        else v = (kk <= c) ? T[i][k] * rsd[c] : 0.0;
        rinv_p[c * LP + kk] = static_cast<TQ>(v);
      }
  }
  if (r_out) {
    if (a0 < LP && b0 < LP) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) Ufull[(a0 + i) * LP + b0 + k] = U[i][k];
    }
    __syncthreads();
    for (int idx = tid; idx < LP * LP; idx += kCholThreads) {
      int a = idx / LP, b = idx - (idx / LP) * LP;
      double v;
      if (a >= l || b >= l) v = (a == b) ? 1.0 : 0.0;
      else if (b < a || rsd[a] == 0.0) v = 0.0;
      else if (!r_prev) v = Ufull[a * LP + b] * rsd[a];
      else {
        v = 0.0;
        for (int k = a; k <= b; ++k) v += Ufull[a * LP + k] * r_prev[k * LP + b];
        v *= rsd[a];
      }
      r_out[idx] = v;
    }
  }
}

template <typename TQ>
hipError_t launch_chol(const double* g, int64_t ldg, int l, int LP, double tau_rel, TQ* rinv_p, double* r_out,
                       const double* r_prev, double* scratch, int* flags, hipStream_t s) {
  if (l < 1 || l > 1024) return hipErrorInvalidValue;
  if (LP <= 128) {
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_reg_kernel<TQ>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    size_t sh = r_out ? (size_t)LP * LP * sizeof(double) : 0;
    hipLaunchKernelGGL((chol_reg_kernel<TQ>), dim3(1), dim3(kCholThreads), sh, s, g, ldg, l, LP, tau_rel, rinv_p,
                       r_out, r_prev, flags);
  } else {
    if (!scratch) return hipErrorInvalidValue;
    return launch_chol_blocked<TQ>(g, ldg, l, LP, tau_rel, rinv_p, r_out, r_prev, scratch, flags, s);
  }
  return hipGetLastError();
}

template hipError_t launch_chol<float>(const double*, int64_t, int, int, double, float*, double*, const double*,
                                       double*, int*, hipStream_t);
template hipError_t launch_chol<double>(const double*, int64_t, int, int, double, double*, double*, const double*,
                                        double*, int*, hipStream_t);

}  // namespace rsvd
