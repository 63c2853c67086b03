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
// floor(l/2) disjoint pairs, processed in parallel by groups of 16 lanes (64
// pairs at once in a 1024-thread block); l-1 (or l) rounds make a sweep.
// Sweeps repeat until no pair needs a rotation (|x_p . x_q| <= tol * ||x_p||
// ||x_q||); after a sweep with few rotations that test is first made on all
// pairs at once from X^T X, which spares the sweep that would rotate nothing.  A column whose norm is at most tol * ||X||_F is numerically zero
// (rank deficiency, below what the stopping test can resolve against the
// other columns): it takes no rotation, and it is returned as sigma = 0 with a
// zero u_hat column, as an exactly zero column is.  A rotation only ever
// shrinks the smaller column of its pair, so such a column stays below the
// bound, and the rounding-level columns of a rank-deficient X no longer need
// the many sweeps it takes to make them mutually orthogonal.  The round is
// bound by instruction issue on one CU, so it is kept
// lean: the squared norms are computed at the start of a sweep and then
// updated exactly as the rotation changes them (||x_p||^2 - t g, ||x_q||^2 +
// t g), so a pair only forms its dot product; the reductions use DPP lane
// moves; the rotation comes from hardware reciprocal and reciprocal-square-root estimates, each
// refined by two Newton steps; a lane holds pairs of consecutive rows (16-byte LDS
// accesses) and the rows past l are zero, so no access is guarded.  Results are sorted by
// descending sigma and each u_hat column is signed so that its entry of
// largest magnitude (lowest index on ties) is positive.
#include "internal.hpp"

namespace rsvd {

__device__ __forceinline__ int rr_player(int pos, int round, int le) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (le - 1);
}

// Lanes per column pair (16: four pairs per wave; eight lanes per pair, which issues the rotation's own
// arithmetic once per eight pairs, measured 10 % slower at l = 110: fewer waves hide less of its latency).
constexpr int kPairLanes = 16;

// Value of the lane chosen by a DPP pattern (applied to both halves of the double).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each aligned group of kPairLanes lanes: lane ^ 1, lane ^ 2 (quad permutes), then the mirror image
// within 8 lanes (and within 16 for groups of 16), each of which pairs a lane with one of the other half.
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  if constexpr (kPairLanes == 16) v += dpp_f64<0x140>(v);   // row_mirror
  return v;
}

// 1/x and 1/sqrt(x) for finite x > 0: the hardware estimate refined by two Newton steps (within a few
// units in the last place, against about ten instructions more for the correctly rounded forms).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);   // y += y (1 - x y^2) / 2
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// Norms, order, signs and outputs of the converged columns: sigma descending, u_hat = x / sigma signed so
// that its entry of largest magnitude (lowest index on ties) is positive, v_hat = u_hat / sigma; a column
// with squared norm at most thr2 (numerically zero) gives sigma = 0 and zero vectors.  Column p of X is at
// xs[p*LX + i]; the outputs have leading dimension LP.  Columns p0 .. p1-1 are written (all by default); every
// caller computes all norms and ranks the same way, so workgroups that split the columns agree on them.
template <typename TU>
__device__ void jacobi_epilogue(const double* xs, int LX, int l, int LP, double thr2, double* nrm, int* rnk,
                                double* __restrict__ sigma, double* __restrict__ uhat_d, TU* __restrict__ uhat_p,
                                TU* __restrict__ vhat_p, int p0 = 0, int p1 = -1) {
  if (p1 < 0) p1 = LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  for (int p = w; p < l; p += nw) {
    double s = 0.0;
    for (int i = lane; i < l; i += 64) s += xs[p * LX + i] * xs[p * LX + i];
    s = wave_sum(s);
    if (lane == 0) nrm[p] = s > thr2 ? sqrt(s) : 0.0;
  }
  __syncthreads();
  for (int p = tid; p < l; p += nt) {
    int r = 0;
    double v = nrm[p];
    for (int q = 0; q < l; ++q) r += (nrm[q] > v) || (nrm[q] == v && q < p);
    rnk[p] = r;
  }
  __syncthreads();
  for (int p = p0 + w; p < p1; p += nw) {
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
      double a = fabs(xs[p * LX + i]);
      if (a > best) { best = a; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    double sg = xs[p * LX + bi] < 0.0 ? -1.0 : 1.0;
    double sv = nrm[p];
    int j = rnk[p];
    double inv = sv > 0.0 ? sg / sv : 0.0;
    double inv2 = sv > 0.0 ? inv / sv : 0.0;
    for (int i = lane; i < LP; i += 64) {
      double x = (i < l) ? xs[p * LX + i] : 0.0;
      uhat_d[(int64_t)j * LP + i] = x * inv;
      if (uhat_p) uhat_p[(int64_t)j * LP + i] = static_cast<TU>(x * inv);
      if (vhat_p) vhat_p[(int64_t)j * LP + i] = static_cast<TU>(x * inv2);
    }
    if (lane == 0) sigma[j] = sv;
  }
}

template <typename TU, int NH>
__device__ __forceinline__ void jacobi_body(const double* __restrict__ R, int l, int LP, double tol, int max_sweeps,
                                            double* __restrict__ sigma, double* __restrict__ uhat_d,
                                            TU* __restrict__ uhat_p, TU* __restrict__ vhat_p,
                                            int* __restrict__ flags) {
  // A lane of a pair group holds rows 2 (sub + kPairLanes h) and the next one, h < NV; LX = 32 NH >= LP.
  constexpr int LX = 32 * NH;
  constexpr int NV = LX / (2 * kPairLanes);   // double2 of a column per lane
  extern __shared__ double2 smem2[];   // 16-byte aligned: accessed as double2
  double* xs = reinterpret_cast<double*>(smem2);   // column p of X = row p of R, at xs[p*LX + i]; rows l .. LX-1 zero
  __shared__ double nrm[1024];
  __shared__ double nrm2[1024];   // squared column norms, kept current through the sweep
  __shared__ int rnk[1024];
  __shared__ int rotated;
  __shared__ int nrot_sh[2];   // rotations of the sweep, by sweep parity
  __shared__ int need_sh;      // the all-pairs test found a pair to rotate
  __shared__ double thr2_sh;   // tol^2 ||X||_F^2: squared norm at or below which a column is numerically zero
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const int slot = tid / kPairLanes, sub = tid % kPairLanes, nslots = nt / kPairLanes;

  for (int idx = tid; idx < l * LX; idx += nt) {
    int p = idx / LX, i = idx - (idx / LX) * LX;
    xs[p * LX + i] = (i < l) ? R[(int64_t)p * LP + i] : 0.0;
  }
  const int le = l + (l & 1);
  const int m1 = le - 1;
  const int npairs = le / 2;
  const double tol2 = tol * tol;
  int sweep = 0;
  bool converged = (l < 2);
  if (tid == 0) {
    thr2_sh = 0.0;
    nrot_sh[0] = nrot_sh[1] = 0;
  }
  for (; sweep < max_sweeps && !converged; ++sweep) {
    __syncthreads();
    const int prev_rot = nrot_sh[(sweep + 1) & 1];   // the previous sweep's rotations
    if (tid == 0) {
      rotated = 0;
      nrot_sh[sweep & 1] = 0;
      need_sh = 0;
    }
    for (int p = w; p < l; p += nw) {
      double ss = 0.0;
      for (int i = lane; i < l; i += 64) ss += xs[p * LX + i] * xs[p * LX + i];
      ss = wave_sum(ss);
      if (lane == 0) nrm2[p] = ss;
    }
    __syncthreads();
    if (sweep == 0) {
      // ||X||_F^2 (invariant under the rotations), summed in column order
      if (tid == 0) {
        double f = 0.0;
        for (int p = 0; p < l; ++p) f += nrm2[p];
        thr2_sh = tol2 * f;
      }
      __syncthreads();
    }
    const double thr2 = thr2_sh;
    // After a sweep that rotated at most a quarter of the pairs, the next one often rotates none.  A sweep
    // that rotates none tests every pair on the unchanged X, so the same test applied at once to X^T X
    // (upper 16 x 16 tiles on the FP64 MFMA, the squared norms of this sweep on the diagonal) ends the
    // iteration without it; the Gram's entries differ from the pair groups' dot products only in the order of
    // summation.  Lane (ci, g) supplies rows 16 s + 4 g + e of its column for MFMA step e; accumulator
    // element r of lane L is G(16 ti + L / 16 + 4 r, 16 tj + L % 16).
    if (sweep > 0 && 4 * prev_rot <= l * (l - 1) / 2) {
      const int nt16 = (l + 15) / 16;
      const int ntile = nt16 * (nt16 + 1) / 2;
      const int ci = lane & 15, g = lane >> 4;
      const int rows16 = nt16 * 16;   // rows l .. rows16 - 1 of X are zero
      for (int tix = w; tix < ntile; tix += nw) {
        int ti = 0, rem = tix;
        while (rem >= nt16 - ti) {
          rem -= nt16 - ti;
          ++ti;
        }
        const int tj = ti + rem;
        const double* xa = xs + min(16 * ti + ci, l - 1) * LX + 4 * g;
        const double* xb = xs + min(16 * tj + ci, l - 1) * LX + 4 * g;
        f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int r0 = 0; r0 < rows16; r0 += 16) {
          const double2 a0 = *reinterpret_cast<const double2*>(xa + r0);
          const double2 a1 = *reinterpret_cast<const double2*>(xa + r0 + 2);
          const double2 b0 = *reinterpret_cast<const double2*>(xb + r0);
          const double2 b1 = *reinterpret_cast<const double2*>(xb + r0 + 2);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b0.x, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b0.y, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1.x, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b1.y, acc, 0, 0, 0);
        }
        bool need = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int p = 16 * ti + (lane >> 4) + 4 * r, q = 16 * tj + (lane & 15);
          if (p < q && q < l) {
            const double al = nrm2[p], be = nrm2[q], ga = acc[r];
            need = need || (al > thr2 && be > thr2 && ga * ga > tol2 * (al * be));
          }
        }
        if (need) need_sh = 1;
      }
      __syncthreads();
      if (need_sh == 0) {   // uniform
        converged = true;
        break;
      }
    }
    int my_rot = 0;
    for (int round = 0; round < m1; ++round) {
      for (int pi = slot; pi < npairs; pi += nslots) {
        // circle method: position 0 stays, the others advance by one each round
        int a = pi - 1 + round;
        a = a >= m1 ? a - m1 : a;
        const int p = pi == 0 ? 0 : 1 + a;
        int b = le - 2 - pi + round;
        b = b >= m1 ? b - m1 : b;
        const int q = 1 + b;
        if (p >= l || q >= l) continue;   // the bye of an odd l (uniform within the pair group)
        double2* xp = reinterpret_cast<double2*>(xs + p * LX) + sub;
        double2* xq = reinterpret_cast<double2*>(xs + q * LX) + sub;
        double2 av[NV], bv[NV];
        double ga = 0.0;
#pragma unroll
        for (int h = 0; h < NV; ++h) {
          av[h] = xp[h * kPairLanes];
          bv[h] = xq[h * kPairLanes];
        }
#pragma unroll
        for (int h = 0; h < NV; ++h) ga += av[h].x * bv[h].x + av[h].y * bv[h].y;
        ga = group_sum(ga);
        const double al = nrm2[p], be = nrm2[q];
        if (al > thr2 && be > thr2 && ga * ga > tol2 * (al * be)) {
          // t = tan of the angle zeroing the off-diagonal of [[al, ga], [ga, be]] (the smaller root)
          const double d = be - al;
          const double h2 = d * d + 4.0 * ga * ga;
          const double hyp = h2 * rsq_nr(h2);                                 // sqrt(h2)
          const double t = (2.0 * ga) * rcp_nr(d >= 0.0 ? d + hyp : d - hyp);  // |t| <= 1
          const double c = rsq_nr(1.0 + t * t);
          const double s = c * t;
#pragma unroll
          for (int h = 0; h < NV; ++h) {
            xp[h * kPairLanes] = make_double2(c * av[h].x - s * bv[h].x, c * av[h].y - s * bv[h].y);
            xq[h * kPairLanes] = make_double2(s * av[h].x + c * bv[h].x, s * av[h].y + c * bv[h].y);
          }
          if (sub == 0) {
            rotated = 1;
            ++my_rot;
            nrm2[p] = al - t * ga;
            nrm2[q] = be + t * ga;
          }
        }
      }
      __syncthreads();
    }
    if (my_rot) atomicAdd(&nrot_sh[sweep & 1], my_rot);
    converged = (rotated == 0);
  }
  if (tid == 0) {
    if (!converged) atomicAdd(&flags[2], 1);
    atomicMax(&flags[3], sweep);
  }
  __syncthreads();

  jacobi_epilogue<TU>(xs, LX, l, LP, thr2_sh, nrm, rnk, sigma, uhat_d, uhat_p, vhat_p);
}

template <typename TU, int NH>
__global__ __launch_bounds__(1024) void jacobi_kernel(const double* __restrict__ R, int l, int LP, double tol,
                                                       int max_sweeps, double* __restrict__ sigma,
                                                       double* __restrict__ uhat_d, TU* __restrict__ uhat_p,
                                                       TU* __restrict__ vhat_p, int* __restrict__ flags) {
  jacobi_body<TU, NH>(R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, flags);
}

// Two independent problems of the same size in one launch, one workgroup each.
template <typename TU, int NH>
__global__ __launch_bounds__(1024) void jacobi2_kernel(JacobiProblem<TU> a, JacobiProblem<TU> b, int l, int LP,
                                                        double tol, int max_sweeps, int* __restrict__ flags) {
  const JacobiProblem<TU>& p = blockIdx.x == 0 ? a : b;
  jacobi_body<TU, NH>(p.R, l, LP, tol, max_sweeps, p.sigma, p.uhat_d, p.uhat_p, p.vhat_p, flags);
}

// Columns per workgroup of the epilogue of the block form (one per wave of 1024 threads); each workgroup
// recomputes all norms and ranks (a read of X from L2) and writes its own columns.
constexpr int kFinishCols = 16;

template <typename TU>
__global__ __launch_bounds__(1024) void jacobi_finish_kernel(const double* __restrict__ xs, int l, int LP,
                                                              const double* __restrict__ thr2,
                                                              double* __restrict__ sigma, double* __restrict__ uhat_d,
                                                              TU* __restrict__ uhat_p, TU* __restrict__ vhat_p) {
  __shared__ double nrm[1024];
  __shared__ int rnk[1024];
  const int p0 = blockIdx.x * kFinishCols;   // this workgroup's columns (one per wave)
  jacobi_epilogue<TU>(xs, LP, l, LP, *thr2, nrm, rnk, sigma, uhat_d, uhat_p, vhat_p, p0, min(LP, p0 + kFinishCols));
}

template <typename TU>
hipError_t jacobi_epilogue_launch(const double* xs, int ldx, int l, int LP, const double* thr2, double* sigma,
                                  double* uhat_d, TU* uhat_p, TU* vhat_p, hipStream_t s) {
  if (ldx != LP) return hipErrorInvalidValue;
  hipLaunchKernelGGL((jacobi_finish_kernel<TU>), dim3((unsigned)((LP + kFinishCols - 1) / kFinishCols)), dim3(1024), 0,
                     s, xs, l, LP, thr2, sigma, uhat_d, uhat_p, vhat_p);
  return hipGetLastError();
}
template hipError_t jacobi_epilogue_launch<float>(const double*, int, int, int, const double*, double*, double*,
                                                  float*, float*, hipStream_t);
template hipError_t jacobi_epilogue_launch<double>(const double*, int, int, int, const double*, double*, double*,
                                                   double*, double*, hipStream_t);

template <typename TU>
hipError_t launch_jacobi(const double* R, int l, int LP, double tol, int max_sweeps, double* sigma, double* uhat_d,
                         TU* uhat_p, TU* vhat_p, double* scratch, int* flags, hipStream_t s) {
  if (l < 1 || l > 1024) return hipErrorInvalidValue;
  if (LP <= 128) {
    // rows held in LDS padded to a multiple of 32 (pairs of rows per lane, kPairLanes lanes per pair)
    const int nh = (LP + 31) / 32;
    static bool attr_set = false;
    if (!attr_set) {
      const void* fns[4] = {reinterpret_cast<const void*>(&jacobi_kernel<TU, 1>),
                            reinterpret_cast<const void*>(&jacobi_kernel<TU, 2>),
                            reinterpret_cast<const void*>(&jacobi_kernel<TU, 3>),
                            reinterpret_cast<const void*>(&jacobi_kernel<TU, 4>)};
      for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
        if (e != hipSuccess) return e;
      }
      attr_set = true;
    }
    size_t sh = (size_t)LP * (32 * nh) * sizeof(double);
    switch (nh) {
      case 1: hipLaunchKernelGGL((jacobi_kernel<TU, 1>), dim3(1), dim3(1024), sh, s, R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, flags); break;
      case 2: hipLaunchKernelGGL((jacobi_kernel<TU, 2>), dim3(1), dim3(1024), sh, s, R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, flags); break;
      case 3: hipLaunchKernelGGL((jacobi_kernel<TU, 3>), dim3(1), dim3(1024), sh, s, R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, flags); break;
      default: hipLaunchKernelGGL((jacobi_kernel<TU, 4>), dim3(1), dim3(1024), sh, s, R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, flags); break;
    }
  } else {
    return launch_jacobi_blocked<TU>(R, l, LP, tol, max_sweeps, sigma, uhat_d, uhat_p, vhat_p, scratch, flags, s);
  }
  return hipGetLastError();
}

template <typename TU>
hipError_t launch_jacobi2(const JacobiProblem<TU>& a, const JacobiProblem<TU>& b, int l, int LP, double tol,
                          int max_sweeps, int* flags, hipStream_t s) {
  if (l < 1 || LP > 128 || LP < l) return hipErrorInvalidValue;
  const int nh = (LP + 31) / 32;
  static bool attr_set = false;
  if (!attr_set) {
    const void* fns[4] = {reinterpret_cast<const void*>(&jacobi2_kernel<TU, 1>),
                          reinterpret_cast<const void*>(&jacobi2_kernel<TU, 2>),
                          reinterpret_cast<const void*>(&jacobi2_kernel<TU, 3>),
                          reinterpret_cast<const void*>(&jacobi2_kernel<TU, 4>)};
    for (const void* f : fns) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
      if (e != hipSuccess) return e;
    }
    attr_set = true;
  }
  const size_t sh = (size_t)LP * (32 * nh) * sizeof(double);
  switch (nh) {
    case 1: hipLaunchKernelGGL((jacobi2_kernel<TU, 1>), dim3(2), dim3(1024), sh, s, a, b, l, LP, tol, max_sweeps, flags); break;
    case 2: hipLaunchKernelGGL((jacobi2_kernel<TU, 2>), dim3(2), dim3(1024), sh, s, a, b, l, LP, tol, max_sweeps, flags); break;
    case 3: hipLaunchKernelGGL((jacobi2_kernel<TU, 3>), dim3(2), dim3(1024), sh, s, a, b, l, LP, tol, max_sweeps, flags); break;
    default: hipLaunchKernelGGL((jacobi2_kernel<TU, 4>), dim3(2), dim3(1024), sh, s, a, b, l, LP, tol, max_sweeps, flags); break;
  }
  return hipGetLastError();
}
template hipError_t launch_jacobi2<float>(const JacobiProblem<float>&, const JacobiProblem<float>&, int, int, double,
                                          int, int*, hipStream_t);
template hipError_t launch_jacobi2<double>(const JacobiProblem<double>&, const JacobiProblem<double>&, int, int,
                                           double, int, int*, hipStream_t);

template hipError_t launch_jacobi<float>(const double*, int, int, double, int, double*, double*, float*, float*,
                                         double*, int*, hipStream_t);
template hipError_t launch_jacobi<double>(const double*, int, int, double, int, double*, double*, double*, double*,
                                          double*, int*, hipStream_t);

}  // namespace rsvd
