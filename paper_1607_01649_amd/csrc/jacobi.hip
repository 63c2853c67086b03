// SVD of the small l x l factor in FP64 by one-sided (Hestenes) Jacobi, in
// one workgroup for l <= 128 (larger l: the block form in blocked.hip).
//
// Stage B (Section 3) needs the SVD of B = Q^T A (l x n).  The library first
// reduces B^T = Q_B R (CholeskyQR2 in FP64), so B = R^T Q_B^T and the SVD of
// the l x l matrix X = R^T gives U_hat directly: rotating the columns of X
// until they are mutually orthogonal yields X J = U_hat diag(sigma), hence
// sigma_p = ||x_p|| and u_hat_p = x_p / sigma_p, with no need to accumulate J.
// The right factor is then recovered as V = B^T U_hat diag(sigma)^-1 by the
// lift kernel.
//
// Pairs are visited in round-robin ("circle method") order: each round holds
// floor(l/2) disjoint pairs, processed in parallel by groups of 8 lanes (128
// pairs at once in a 1024-thread block); l-1 (or l) rounds make a sweep.  Sweeps repeat until no pair needs a
// rotation (|x_p . x_q| <= tol * ||x_p|| ||x_q||).  Results are sorted by
// descending sigma and each u_hat column is signed so that its entry of
// largest magnitude (lowest index on ties) is positive.
#include "internal.hpp"

namespace rsvd {

__device__ __forceinline__ int rr_player(int pos, int round, int le) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (le - 1);
}

// Lanes per column pair.  The kernel is VALU-bound on one CU, so packing
// several pairs into each wave (fewer waves per round) is what pays.
constexpr int kPairLanes = 8;

// Reduction over the lanes of one pair group.
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = kPairLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kPairLanes);
  return v;
}

// Norms, order, signs and outputs of the converged columns (column p of X at
// xs[p*LP + i]): sigma descending, u_hat = x / sigma signed so that its entry
// of largest magnitude (lowest index on ties) is positive, v_hat = u_hat / sigma.
template <typename TU>
__device__ void jacobi_epilogue(const double* xs, int l, int LP, double* nrm, int* rnk, double* __restrict__ sigma,
                                double* __restrict__ uhat_d, TU* __restrict__ uhat_p, TU* __restrict__ vhat_p) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  for (int p = w; p < l; p += nw) {
    double s = 0.0;
    for (int i = lane; i < l; i += 64) s += xs[p * LP + i] * xs[p * LP + i];
    s = wave_sum(s);
    if (lane == 0) nrm[p] = sqrt(s);
  }
  __syncthreads();
  for (int p = tid; p < l; p += nt) {
    int r = 0;
    double v = nrm[p];
    for (int q = 0; q < l; ++q) r += (nrm[q] > v) || (nrm[q] == v && q < p);
    rnk[p] = r;
  }
  __syncthreads();
  for (int p = w; p < LP; p += nw) {
    if (p >= l) {   // padding: zero column at the same index
      for (int i = lane; i < LP; i += 64) {
        uhat_d[(int64_t)p * LP + i] = 0.0;
        if (uhat_p) uhat_p[(int64_t)p * LP + i] = TU(0);
        if (vhat_p) vhat_p[(int64_t)p * LP + i] = TU(0);
      }
      if (lane == 0) sigma[p] = 0.0;
      continue;
    }
    // index of the entry of largest magnitude, lowest index on ties
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < l; i += 64) {
      double a = fabs(xs[p * LP + i]);
      if (a > best) { best = a; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    double sg = xs[p * LP + bi] < 0.0 ? -1.0 : 1.0;
    double sv = nrm[p];
    int j = rnk[p];
    double inv = sv > 0.0 ? sg / sv : 0.0;
    double inv2 = sv > 0.0 ? inv / sv : 0.0;
    for (int i = lane; i < LP; i += 64) {
      double x = (i < l) ? xs[p * LP + i] : 0.0;
      uhat_d[(int64_t)j * LP + i] = x * inv;
      if (uhat_p) uhat_p[(int64_t)j * LP + i] = static_cast<TU>(x * inv);
      if (vhat_p) vhat_p[(int64_t)j * LP + i] = static_cast<TU>(x * inv2);
    }
    if (lane == 0) sigma[j] = sv;
  }
}

template <typename TU>
__global__ __launch_bounds__(1024) void jacobi_kernel(const double* __restrict__ R, int l, int LP, double tol,
                                                       int max_sweeps, double* __restrict__ sigma,
                                                       double* __restrict__ uhat_d, TU* __restrict__ uhat_p,
                                                       TU* __restrict__ vhat_p, int* __restrict__ flags) {
  extern __shared__ double smem[];
  double* xs = smem;   // column p of X = row p of R, at xs[p*LP + i]
  __shared__ double nrm[1024];
  __shared__ int rnk[1024];
  __shared__ int rotated;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const int slot = tid / kPairLanes, sub = tid % kPairLanes, nslots = nt / kPairLanes;

  for (int idx = tid; idx < l * l; idx += nt) {
    int p = idx / l, i = idx - (idx / l) * l;
    xs[p * LP + i] = R[(int64_t)p * LP + i];
  }
  const int le = l + (l & 1);
  const int npairs = le / 2;
  int sweep = 0;
  bool converged = (l < 2);
  for (; sweep < max_sweeps && !converged; ++sweep) {
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < le - 1; ++round) {
      for (int pi = slot; pi < npairs; pi += nslots) {
        int p = rr_player(pi, round, le), q = rr_player(le - 1 - pi, round, le);
        if (p >= l || q >= l) continue;   // uniform within the pair group
        double* xp = xs + p * LP;
        double* xq = xs + q * LP;
        // the lane's slice of both columns, loaded at once (unrolled, predicated) and kept for the rotation
        constexpr int NI = 128 / kPairLanes;
        double av[NI], bv[NI];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
          const int i = sub + u * kPairLanes;
          av[u] = (i < l) ? xp[i] : 0.0;
          bv[u] = (i < l) ? xq[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
          al += av[u] * av[u]; be += bv[u] * bv[u]; ga += av[u] * bv[u];
        }
        al = group_sum(al); be = group_sum(be); ga = group_sum(ga);
        if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          double zeta = (be - al) / (2.0 * ga);
          double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t);
          double s = c * t;
#pragma unroll
          for (int u = 0; u < NI; ++u) {
            const int i = sub + u * kPairLanes;
            if (i < l) {
              xp[i] = c * av[u] - s * bv[u];
              xq[i] = s * av[u] + c * bv[u];
            }
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    converged = (rotated == 0);
  }
  if (tid == 0) {
    if (!converged) atomicAdd(&flags[2], 1);
    atomicMax(&flags[3], sweep);
  }
  __syncthreads();

  jacobi_epilogue<TU>(xs, l, LP, nrm, rnk, sigma, uhat_d, uhat_p, vhat_p);
}

template <typename TU>
__global__ __launch_bounds__(1024) void jacobi_finish_kernel(const double* __restrict__ xs, int l, int LP,
                                                              double* __restrict__ sigma, double* __restrict__ uhat_d,
                                                              TU* __restrict__ uhat_p, TU* __restrict__ vhat_p) {
  __shared__ double nrm[1024];
  __shared__ int rnk[1024];
  jacobi_epilogue<TU>(xs, l, LP, nrm, rnk, sigma, uhat_d, uhat_p, vhat_p);
}

template <typename TU>
hipError_t jacobi_epilogue_launch(const double* xs, int ldx, int l, int LP, double* sigma, double* uhat_d,
                                  TU* uhat_p, TU* vhat_p, hipStream_t s) {
  if (ldx != LP) return hipErrorInvalidValue;
  hipLaunchKernelGGL((jacobi_finish_kernel<TU>), dim3(1), dim3(1024), 0, s, xs, l, LP, sigma, uhat_d, uhat_p,
                     vhat_p);
  return hipGetLastError();
}
template hipError_t jacobi_epilogue_launch<float>(const double*, int, int, int, double*, double*, float*, float*,
                                                  hipStream_t);
template hipError_t jacobi_epilogue_launch<double>(const double*, int, int, int, double*, double*, double*, double*,
                                                   hipStream_t);

template <typename TU>
hipError_t launch_jacobi(const double* R, int l, int LP, double tol, int max_sweeps, double* sigma, double* uhat_d,
                         TU* uhat_p, TU* vhat_p, double* scratch, int* flags, hipStream_t s) {
  if (l < 1 || l > 1024) return hipErrorInvalidValue;
  if (LP <= 128) {
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel<TU>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    size_t sh = (size_t)LP * LP * sizeof(double);
    hipLaunchKernelGGL((jacobi_kernel<TU>), dim3(1), dim3(1024), sh, s, R, l, LP, tol, max_sweeps, sigma,
                       uhat_d, uhat_p, vhat_p, flags);
  } else {
    return launch_jacobi_blocked<TU>(R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, scratch, flags, s);
  }
  return hipGetLastError();
}

template hipError_t launch_jacobi<float>(const double*, int, int, double, int, double*, double*, float*, float*,
                                         double*, int*, hipStream_t);
template hipError_t launch_jacobi<double>(const double*, int, int, double, int, double*, double*, double*, double*,
                                          double*, int*, hipStream_t);

}  // namespace rsvd
