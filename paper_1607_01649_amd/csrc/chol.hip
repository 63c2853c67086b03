// Cholesky factorisation of the l x l Gram matrix of CholeskyQR, in FP64, in
// one workgroup.
//
// orth(Y) (Section 2.3: any unpivoted orthonormalisation will do) is computed
// as CholeskyQR: G = Y^T Y = R^T R, Q = Y R^-1.  This kernel factors G and at
// the same time builds R^-T by applying every elimination step to an identity
// block (Gauss-Jordan style), so the triangular apply that follows is a plain
// panel product with R^-1 and no sequential back-substitution is needed.
//
// Storage: one LP x LP FP64 array M (LDS when LP <= 128, otherwise global
// scratch): the upper triangle including the diagonal holds R, the strict lower
// triangle holds R^-T; the diagonal of R^-T (1/R_jj) is kept apart.
//
// Numerically dependent columns (pivot <= tau_rel * G_jj) are dropped: row j
// of R becomes e_j and row j of R^-T becomes zero, so column j of Q comes out
// exactly zero and later columns are unaffected.  They are counted in
// flags[1]; a non-finite pivot is counted in flags[0].
#include "internal.hpp"

namespace rsvd {

template <typename TQ, bool USE_LDS>
__global__ __launch_bounds__(1024) void chol_kernel(const double* __restrict__ g, int64_t ldg, int l, int LP,
                                                     double tau_rel, TQ* __restrict__ rinv_p, double* __restrict__ r_out,
                                                     const double* __restrict__ r_prev, double* __restrict__ scratch,
                                                     int* __restrict__ flags) {
  extern __shared__ double smem[];
  double* M = USE_LDS ? smem : scratch;
  __shared__ double dg[1024];      // 1 / R_jj (0 for a dropped column)
  __shared__ double gdiag[1024];   // original diagonal of G
  const int tid = threadIdx.x, nt = blockDim.x;

  for (int idx = tid; idx < l * l; idx += nt) {
    int a = idx / l, b = idx % l;
    M[a * LP + b] = (a <= b) ? g[(int64_t)b * ldg + a] : 0.0;
    if (a == b) gdiag[a] = M[a * LP + a];
  }
  __syncthreads();

  for (int j = 0; j < l; ++j) {
    if (tid == 0) {
      double d = M[j * LP + j];
      double gd = gdiag[j];
      if (!isfinite(d) || !isfinite(gd)) {
        atomicAdd(&flags[0], 1);
        M[j * LP + j] = 1.0;
        dg[j] = 0.0;
      } else if (d <= tau_rel * gd || d <= 0.0) {
        atomicAdd(&flags[1], 1);
        M[j * LP + j] = 1.0;
        dg[j] = 0.0;
      } else {
        double r = sqrt(d);
        M[j * LP + j] = r;
        dg[j] = 1.0 / r;
      }
    }
    __syncthreads();
    const double s = dg[j];
    // row j: R part (b > j) and R^-T part (b < j) scale by 1/R_jj; a dropped
    // column zeroes both.
    for (int b = tid; b < l; b += nt)
      if (b != j) M[j * LP + b] *= s;
    __syncthreads();
    // rows a > j: R trailing update (b >= a) and R^-T update (b <= j).
    const int nrow = l - j - 1;
    for (int idx = tid; idx < nrow * l; idx += nt) {
      int a = j + 1 + idx / l, b = idx % l;
      double rja = M[j * LP + a];
      if (b >= a || b < j) M[a * LP + b] -= rja * M[j * LP + b];
      else if (b == j) M[a * LP + j] -= rja * s;
    }
    __syncthreads();
  }

  // R^-1 in panel layout: rinv_p[c*LP + k] = R^-1(k, c) = R^-T(c, k).
  for (int idx = tid; idx < LP * LP; idx += nt) {
    int c = idx / LP, k = idx % LP;
    double v;
    if (c >= l || k >= l) v = (c == k) ? 1.0 : 0.0;
    else if (k < c) v = M[c * LP + k];
    else if (k == c) v = dg[c];
    else v = 0.0;
    rinv_p[idx] = static_cast<TQ>(v);
  }
  if (r_out) {
    for (int idx = tid; idx < LP * LP; idx += nt) {
      int a = idx / LP, b = idx % LP;
      double v;
      if (a >= l || b >= l) v = (a == b) ? 1.0 : 0.0;
      else if (b < a || dg[a] == 0.0) v = 0.0;   // a dropped column leaves a zero row of R
      else if (!r_prev) v = M[a * LP + b];
      else {
        v = 0.0;
        for (int k = a; k <= b; ++k) v += M[a * LP + k] * r_prev[k * LP + b];
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
    hipLaunchKernelGGL((chol_kernel<TQ, true>), dim3(1), dim3(1024), sh, s, g, ldg, l, LP, tau_rel, rinv_p, r_out,
                       r_prev, scratch, flags);
  } else {
    hipLaunchKernelGGL((chol_kernel<TQ, false>), dim3(1), dim3(1024), 0, s, g, ldg, l, LP, tau_rel, rinv_p, r_out,
                       r_prev, scratch, flags);
  }
  return hipGetLastError();
}

template hipError_t launch_chol<float>(const double*, int64_t, int, int, double, float*, double*, const double*,
                                       double*, int*, hipStream_t);
template hipError_t launch_chol<double>(const double*, int64_t, int, int, double, double*, double*, const double*,
                                        double*, int*, hipStream_t);

}  // namespace rsvd
