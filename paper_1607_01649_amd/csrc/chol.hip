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
// Storage: one LP x LP FP64 array M (LDS when LP <= 128, else global
// scratch): the upper triangle including the diagonal holds U, the strict
// lower triangle holds T (whose unit diagonal is implicit).  Each thread owns
// the entries idx = tid + 1024 u of the l x l block.
//
// Numerically dependent columns (pivot <= tau_rel * G_jj) are dropped: they
// take no part in later eliminations, row j of R and column j of R^-1 come out
// zero (so column j of Q is exactly zero).  Counted in flags[1]; a non-finite
// pivot is counted in flags[0].
#include "internal.hpp"

namespace rsvd {

constexpr int kCholThreads = 1024;
constexpr int kCholOwn = 16;   // entries per thread kept in registers when l <= 128

template <typename TQ, bool USE_LDS>
__global__ __launch_bounds__(kCholThreads) void chol_kernel(const double* __restrict__ g, int64_t ldg, int l, int LP,
                                                             double tau_rel, TQ* __restrict__ rinv_p,
                                                             double* __restrict__ r_out,
                                                             const double* __restrict__ r_prev,
                                                             double* __restrict__ scratch, int* __restrict__ flags) {
  extern __shared__ double smem[];
  double* M = USE_LDS ? smem : scratch;
  __shared__ double gdiag[1024];   // original diagonal of G
  __shared__ double rsd[1024];     // 1/sqrt(d_j), 0 for a dropped column
  const int tid = threadIdx.x;
  const int ll = l * l;

  for (int idx = tid; idx < ll; idx += kCholThreads) {
    int a = idx / l, b = idx - (idx / l) * l;
    double v = (a <= b) ? g[(int64_t)b * ldg + a] : 0.0;
    M[a * LP + b] = v;
    if (a == b) gdiag[a] = v;
  }
  __syncthreads();

  int own_a[kCholOwn], own_b[kCholOwn];
  const int nown = USE_LDS ? (ll - tid + kCholThreads - 1) / kCholThreads : 0;
  if (USE_LDS) {
#pragma unroll
    for (int u = 0; u < kCholOwn; ++u) {
      int idx = tid + kCholThreads * u;
      own_a[u] = idx < ll ? idx / l : -1;
      own_b[u] = idx < ll ? idx - (idx / l) * l : 0;
    }
  }

  int bad = 0, dropped = 0;
  for (int j = 0; j < l; ++j) {
    const double d = M[j * LP + j];
    const double gd = gdiag[j];
    const bool nonfinite = !isfinite(d) || !isfinite(gd);
    const bool drop = nonfinite || !(d > tau_rel * gd) || !(d > 0.0);
    bad += nonfinite;
    dropped += (drop && !nonfinite);
    if (!drop) {
      const double invd = 1.0 / d;
      if (USE_LDS) {
#pragma unroll
        for (int u = 0; u < kCholOwn; ++u) {
          if (u >= nown) break;
          int a = own_a[u], b = own_b[u];
          if (a <= j) continue;
          double f = M[j * LP + a] * invd;
          if (b >= a) M[a * LP + b] -= f * M[j * LP + b];
          else if (b < j) M[a * LP + b] -= f * M[j * LP + b];
          else if (b == j) M[a * LP + b] = -f;
        }
      } else {
        for (int idx = tid; idx < ll; idx += kCholThreads) {
          int a = idx / l, b = idx - (idx / l) * l;
          if (a <= j) continue;
          double f = M[j * LP + a] * invd;
          if (b >= a) M[a * LP + b] -= f * M[j * LP + b];
          else if (b < j) M[a * LP + b] -= f * M[j * LP + b];
          else if (b == j) M[a * LP + b] = -f;
        }
      }
    }
    if (tid == j % kCholThreads) rsd[j] = drop ? 0.0 : 1.0 / sqrt(d);
    __syncthreads();
  }
  if (tid == 0) {
    if (bad) atomicAdd(&flags[0], bad);
    if (dropped) atomicAdd(&flags[1], dropped);
  }

  // R^-1 in panel layout: rinv_p[c*LP + k] = R^-1(k, c) = R^-T(c, k) = T(c, k) / sqrt(d_c).
  for (int idx = tid; idx < LP * LP; idx += kCholThreads) {
    int c = idx / LP, k = idx - (idx / LP) * LP;
    double v;
    if (c >= l || k >= l) v = (c == k) ? 1.0 : 0.0;
    else if (k < c) v = M[c * LP + k] * rsd[c];
    else if (k == c) v = rsd[c];
    else v = 0.0;
    rinv_p[idx] = static_cast<TQ>(v);
  }
  if (r_out) {
    // R(a, b) = U(a, b) / sqrt(d_a); optionally times r_prev (both upper triangular).
    for (int idx = tid; idx < LP * LP; idx += kCholThreads) {
      int a = idx / LP, b = idx - (idx / LP) * LP;
      double v;
      if (a >= l || b >= l) v = (a == b) ? 1.0 : 0.0;
      else if (b < a || rsd[a] == 0.0) v = 0.0;
      else if (!r_prev) v = M[a * LP + b] * rsd[a];
      else {
        v = 0.0;
        for (int k = a; k <= b; ++k) v += M[a * LP + k] * r_prev[k * LP + b];
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
    size_t sh = (size_t)LP * LP * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_kernel<TQ, true>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    hipLaunchKernelGGL((chol_kernel<TQ, true>), dim3(1), dim3(kCholThreads), sh, s, g, ldg, l, LP, tau_rel, rinv_p,
                       r_out, r_prev, scratch, flags);
  } else {
    hipLaunchKernelGGL((chol_kernel<TQ, false>), dim3(1), dim3(kCholThreads), 0, s, g, ldg, l, LP, tau_rel, rinv_p,
                       r_out, r_prev, scratch, flags);
  }
  return hipGetLastError();
}

template hipError_t launch_chol<float>(const double*, int64_t, int, int, double, float*, double*, const double*,
                                       double*, int*, hipStream_t);
template hipError_t launch_chol<double>(const double*, int64_t, int, int, double, double*, double*, const double*,
                                        double*, int*, hipStream_t);

}  // namespace rsvd
