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
// with d_j = U(j, j); the steps are grouped in panels of 16 pivots (below).
// At the end R = D^-1/2 U and R^-T = D^-1/2 T.
//
// Storage: register blocks, l <= 128; larger l goes to the blocked
// multi-workgroup form in blocked.hip.
//
// Numerically dependent columns (pivot <= tau_rel * G_jj) are dropped: they
// take no part in later eliminations, row j of R and column j of R^-1 come out
// zero (so column j of Q is exactly zero).  Counted in flags[1]; a non-finite
// pivot is counted in flags[0].
#include <algorithm>

#include "internal.hpp"

namespace rsvd {

constexpr int kCholThreads = 1024;

// Value of lane `src` (wave-uniform) of a double held in a VGPR.
__device__ __forceinline__ double lane_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int kCholNB = 16;     // pivots per panel
constexpr int kCholPitch = 132; // LDS pitch of a published panel row (16-byte aligned quads)

// l <= 128: thread t owns the 4 x 4 register blocks U[4][4] and T[4][4] of
// rows a0..a0+3 and columns b0..b0+3.  A wave covers a 32 x 32 tile (wave w:
// row band w / 4, column band w % 4), so whole waves skip what is dead for
// them (rows all before the panel, U columns all before it, T columns all
// after it).  U starts as G's upper triangle, T as the identity.
// The pivots are taken in panels P = [p0, p0+16), with three barriers per
// panel instead of one per pivot:
//   1. the owners of the panel rows publish [U(P, :) T(P, :)] to LDS;
//   2. the panel rows are eliminated among themselves pivot by pivot, one
//      lane per column: lanes 0..15 of each of waves 0..3 hold the 16 x 16
//      diagonal block (so the pivot and the pivot row's entries reach every
//      lane of the wave by lane broadcast, with no barrier, and each lane
//      divides its own entry by the pivot meanwhile), the other lanes hold
//      the U columns right of the block and the T columns up to the panel's
//      end;
//   3. every trailing row a takes the panel's pivots at once,
//      [U(a, :) T(a, :)] -= sum_j U(j, a) / d_j [U(j, :) T(j, :)] over the
//      final panel rows, and the panel rows take their final values.
// This is the elimination of one pivot at a time regrouped (each update uses
// the pivot row as it stands after the earlier pivots, as before); only the
// order in which a trailing entry receives the panel's 16 terms changes.
template <typename TQ>
__global__ __launch_bounds__(kCholThreads) void chol_panel_kernel(const double* __restrict__ g, int64_t ldg, int l,
                                                                   int LP, double tau_rel, TQ* __restrict__ rinv_p,
                                                                   double* __restrict__ r_out,
                                                                   const double* __restrict__ r_prev,
                                                                   int* __restrict__ flags) {
  __shared__ double dinvP[kCholNB];                          // 1/d_j, 0 for a dropped pivot
  __shared__ double DblkIn[kCholNB * (kCholNB + 1)];         // diagonal block as published
  __shared__ double Dblk[kCholNB * (kCholNB + 1)];           // eliminated diagonal block (upper)
  __shared__ double gdiag[128];
  __shared__ double rsd[128];     // 1/sqrt(d_j), 0 for a dropped column
  // dynamic LDS: the panel rows [Up | Tp] during the elimination, then (when r_out
  // is wanted) U as LP x LP for the output
  extern __shared__ __align__(16) double chol_dyn[];
  double* Up = chol_dyn;                          // U part of the panel rows
  double* Tp = chol_dyn + kCholNB * kCholPitch;   // T part of the panel rows
  double* Ufull = chol_dyn;
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), ln = tid & 63;   // wave index in a scalar register
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
  for (int p0 = 0; p0 < l; p0 += kCholNB) {
    const int np = min(kCholNB, l - p0), pe = p0 + np;
    // 1. publish the panel rows
    if (a0 + 3 >= p0 && a0 < pe) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = a0 + i;
        if (a >= p0 && a < pe)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int b = b0 + k;
            // Up holds the columns right of the panel (zero elsewhere); the diagonal block
            // goes to DblkIn
            Up[(a - p0) * kCholPitch + b] = (b >= pe) ? U[i][k] : 0.0;
            if (b >= p0 && b < pe) DblkIn[(a - p0) * (kCholNB + 1) + b - p0] = (b >= a) ? U[i][k] : 0.0;
            Tp[(a - p0) * kCholPitch + b] = T[i][k];
          }
      }
    }
    __syncthreads();
    // 2+3. the panel's pivots, one at a time, over all columns of the panel rows.  Waves
    // 0..3 each hold the diagonal block's columns in lanes 0..15 (each wave factors it, so
    // the multipliers come by lane broadcast within the wave) and, in lanes 16..63, the U
    // columns right of the block and the T columns up to the panel's end (48 per wave).
    if (wv < 4) {
      const int c = ln;
      const int nuc = LP - pe;
      const int o = 48 * wv + (c - 16);
      double* colp = nullptr;   // this lane's column of [Up | Tp] (pitch kCholPitch)
      if (c < 16) colp = (c < np) ? DblkIn + c : nullptr;
      else if (o < nuc) colp = Up + pe + o;
      else if (o - nuc < pe) colp = Tp + (o - nuc);
      double col[kCholNB];
      const int pitch = (c < 16) ? kCholNB + 1 : kCholPitch;
#pragma unroll
      for (int a = 0; a < kCholNB; ++a) col[a] = (colp && a < np) ? colp[a * pitch] : 0.0;
      const double gdl = (c < np) ? gdiag[p0 + c] : 0.0;   // lane j: G_jj of pivot j
      const int lim = (c < 16) ? c : kCholNB - 1;   // diagonal-block lanes keep to the upper triangle
#pragma unroll
      for (int j = 0; j < kCholNB; ++j) {
        if (j < np) {
          const double d = lane_f64(col[j], j);
          const double gd = lane_f64(gdl, j);
          const bool nonfinite = !isfinite(d) || !isfinite(gd);
          const bool drop = nonfinite || !(d > tau_rel * gd) || !(d > 0.0);
          // 1/d_j: hardware estimate and two Newton steps
          double r = __builtin_amdgcn_rcp(d);
          r = fma(r, fma(-d, r, 1.0), r);
          r = fma(r, fma(-d, r, 1.0), r);
          const double dinv = drop ? 0.0 : r;
          if (tid == 0) {
            dinvP[j] = dinv;
            bad += nonfinite;
            dropped += (drop && !nonfinite);
          }
          // U(a, c) -= U(j, a) * (U(j, c) / d_j), the pivot row's entries by broadcast
          const double t = col[j] * dinv;
#pragma unroll
          for (int a = j + 1; a < kCholNB; ++a) {
            const double ua = lane_f64(col[j], a);   // U(p0+j, p0+a)
            if (a <= lim) col[a] -= ua * t;
          }
        }
        asm volatile("" ::: "memory");
      }
      if (c < 16) {
        if (wv == 0 && c < np)   // the eliminated diagonal block
#pragma unroll
          for (int a = 0; a < kCholNB; ++a)
            if (a < np) Dblk[a * (kCholNB + 1) + c] = col[a];
      } else if (colp) {
#pragma unroll
        for (int a = 0; a < kCholNB; ++a)
          if (a < np) colp[a * kCholPitch] = col[a];
      }
    }
    __syncthreads();
    // 3. final panel rows; trailing rows take the panel's pivots.  In Up the columns left
    // of pe are zero and in Tp the entries right of each row's diagonal are zero (they
    // stay exactly zero through the elimination), so f, ub and tb below need no masks.
    if (tid < np) rsd[p0 + tid] = dinvP[tid] > 0.0 ? sqrt(dinvP[tid]) : 0.0;
    if (rlast >= p0) {   // uniform over the wave
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = a0 + i;
        if (a >= p0 && a < pe)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int b = b0 + k;
            if (b >= pe) U[i][k] = Up[(a - p0) * kCholPitch + b];
            else if (b >= a) U[i][k] = Dblk[(a - p0) * (kCholNB + 1) + b - p0];
            T[i][k] = Tp[(a - p0) * kCholPitch + b];
          }
      }
      if (rlast >= pe) {
        // U is needed on and above the diagonal, T on and below it
        const bool doU = clast >= pe && (wv >> 2) <= (wv & 3), doT = cfirst < pe && (wv & 3) <= (wv >> 2);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
          const double dj = dinvP[j];   // 0 for a dropped pivot: no elimination
          const double* uj = Up + j * kCholPitch;
          const double* tj = Tp + j * kCholPitch;
          double f[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) f[i] = uj[a0 + i] * dj;
          if (doU) {
            double ub[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) ub[k] = uj[b0 + k];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int k = 0; k < 4; ++k) U[i][k] -= f[i] * ub[k];
          }
          if (doT) {
            double tb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) tb[k] = tj[b0 + k];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int k = 0; k < 4; ++k) T[i][k] -= f[i] * tb[k];
          }
        }
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
    // R = D^-1/2 U, or D^-1/2 U R_prev when the previous pass's factor is given (the product
    // of the two passes of CholeskyQR2): each thread its own 4 x 4 block; k runs over
    // [a0, b0+3], the terms outside [a, b] being exact zeros (U masked left of its diagonal,
    // R_prev upper triangular with identity padding).
    if (a0 < LP && b0 < LP) {
      double acc[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[i][k] = 0.0;
      if (r_prev) {
        const int kend = min(b0 + 3, l - 1);
#pragma unroll 4
        for (int k = a0; k <= kend; ++k) {
          const double2 p01 = *reinterpret_cast<const double2*>(r_prev + (int64_t)k * LP + b0);
          const double2 p23 = *reinterpret_cast<const double2*>(r_prev + (int64_t)k * LP + b0 + 2);
          const double p[4] = {p01.x, p01.y, p23.x, p23.y};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double u = (k >= a0 + i) ? Ufull[(a0 + i) * LP + k] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += u * p[j];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = a0 + i, b = b0 + j;
          double v;
          if (a >= l || b >= l) v = (a == b) ? 1.0 : 0.0;
          else if (b < a || rsd[a] == 0.0) v = 0.0;
          else v = (r_prev ? acc[i][j] : Ufull[a * LP + b]) * rsd[a];
          r_out[a * LP + b] = v;
        }
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
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_panel_kernel<TQ>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    size_t sh = 2 * kCholNB * kCholPitch * sizeof(double);
    if (r_out) sh = std::max(sh, (size_t)LP * LP * sizeof(double));
    hipLaunchKernelGGL((chol_panel_kernel<TQ>), dim3(1), dim3(kCholThreads), sh, s, g, ldg, l, LP, tau_rel, rinv_p,
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
