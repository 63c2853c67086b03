// Multi-workgroup forms of the two small FP64 factorisations for l > 128:
// the Cholesky factorisation (with R^-1) of CholeskyQR's Gram matrix, and the
// one-sided Jacobi SVD of the l x l factor of Stage B.  Both keep the meaning
// of the one-workgroup kernels in chol.hip and jacobi.hip; only the schedule
// changes, so that the work of a step is spread over many compute units.
//
// Cholesky (right-looking, 64 x 64 blocks, working matrix M row-major LB x LB):
//   for each block column J:
//     factor the diagonal block (one workgroup, the same unscaled elimination
//     with the identity block as chol.hip, dependent columns dropped against
//     the original diagonal) -> R_JJ and S_JJ = R_JJ^-1;
//     R_JK = S_JJ^T M_JK for the blocks K > J of the block row;
//     M_KL -= R_JK^T R_JL for J < K <= L.
//   R^-1 by block back-substitution: X_JJ = S_JJ and, for I from the bottom,
//     X_IJ = -S_II sum_{I < K <= J} R_IK X_KJ  (all J > I at once).
// Dropped columns give zero rows of R and zero rows and columns of R^-1, as
// in the one-workgroup kernel.
//
// Jacobi (block one-sided, X = R^T): the columns are split into blocks of W;
// the blocks are paired by the round-robin (circle) ordering, one workgroup
// per pair holds the pair's 2W columns in LDS and runs inner one-sided Jacobi
// sweeps (the same rotation and test as jacobi.hip) over all of its column
// pairs.  A sweep of nbk-1 rounds meets every pair of blocks, hence every
// pair of columns; sweeps repeat until one passes in which no workgroup had to
// rotate in its first inner sweep.
#include "internal.hpp"

namespace rsvd {

constexpr int CB = 64;   // Cholesky block

__global__ void bc_init_kernel(const double* __restrict__ g, int64_t ldg, int l, int LB, double* __restrict__ M,
                               double* __restrict__ gdiag) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)LB * LB) return;
  const int a = (int)(t / LB), b = (int)(t - (t / LB) * LB);
  const double v = (a <= b && b < l) ? g[(int64_t)b * ldg + a] : 0.0;
  M[t] = v;
  if (a == b) gdiag[a] = v;
}

// Diagonal block J (rows/columns j0 .. j0+63) of M: 256 threads, thread t owns the 4 x 4
// register blocks of U and T at rows 4*(t/16), columns 4*(t%16).
__global__ __launch_bounds__(256) void bc_diag_kernel(double* __restrict__ M, int LB, int j0, int l,
                                                      const double* __restrict__ gdiag, double tau,
                                                      double* __restrict__ X, int* __restrict__ flags) {
  __shared__ double urow[2][CB];
  __shared__ double trow[2][CB];
  __shared__ double rs[CB];
  const int tid = threadIdx.x;
  const int a0 = 4 * (tid >> 4), b0 = 4 * (tid & 15);
  const int nv = min(CB, l - j0);
  double U[4][4], T[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = a0 + i, b = b0 + k;
      U[i][k] = (a <= b && b < nv) ? M[(int64_t)(j0 + a) * LB + j0 + b] : 0.0;
      T[i][k] = (a == b) ? 1.0 : 0.0;
    }
  if (a0 == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) { urow[0][b0 + k] = U[0][k]; trow[0][b0 + k] = T[0][k]; }
  }
  if (tid < CB) rs[tid] = 0.0;
  __syncthreads();
  int bad = 0, dropped = 0;
  for (int j = 0; j < nv; ++j) {
    const double* uj = urow[j & 1];
    const double* tj = trow[j & 1];
    const double d = uj[j];
    const double gd = gdiag[j0 + j];
    const bool nonfinite = !isfinite(d) || !isfinite(gd);
    const bool drop = nonfinite || !(d > tau * gd) || !(d > 0.0);
    bad += nonfinite;
    dropped += (drop && !nonfinite);
    if (!drop && a0 + 3 > j) {
      const double invd = 1.0 / d;
      double f[4], ub[4], tb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) f[i] = (a0 + i > j) ? uj[a0 + i] * invd : 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ub[k] = (b0 + k > j) ? uj[b0 + k] : 0.0;
        tb[k] = tj[b0 + k];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          U[i][k] -= f[i] * ub[k];
          T[i][k] -= f[i] * tb[k];
        }
    }
    if (tid == 0) rs[j] = drop ? 0.0 : 1.0 / sqrt(d);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (a0 + i == j + 1 && j + 1 < nv) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          urow[(j + 1) & 1][b0 + k] = U[i][k];
          trow[(j + 1) & 1][b0 + k] = T[i][k];
        }
      }
    __syncthreads();
  }
  if (tid == 0) {
    if (bad) atomicAdd(&flags[0], bad);
    if (dropped) atomicAdd(&flags[1], dropped);
  }
  // R_JJ = D^-1/2 U (upper, in place) and R_JJ^-1 (k, c) = T(c, k) / sqrt(d_c) into X's diagonal block.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = a0 + i, b = b0 + k;
      M[(int64_t)(j0 + a) * LB + j0 + b] = (a <= b) ? U[i][k] * rs[a] : 0.0;
      X[(int64_t)(j0 + b) * LB + j0 + a] = (b <= a) ? T[i][k] * rs[a] : 0.0;
    }
}

// 64 x 64 tile product helper: acc(a, b) += sum_t As[t][a] * Bs[t][b] over the staged tiles
// (ld CB + 1), thread t owning rows 4*(t/16) and columns 4*(t%16).
__device__ __forceinline__ void tile_tn(const double (*As)[CB + 1], const double (*Bs)[CB + 1], int a0, int b0,
                                        double (&acc)[4][4]) {
#pragma unroll 4
  for (int t = 0; t < CB; ++t) {
    double av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = As[t][a0 + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) bv[k] = Bs[t][b0 + k];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[i][k] += av[i] * bv[k];
  }
}

// R_JK = S_JJ^T M_JK for the blocks K = J+1+blockIdx.x.
__global__ __launch_bounds__(256) void bc_panel_kernel(double* __restrict__ M, const double* __restrict__ X, int LB,
                                                       int j0) {
  __shared__ double Ss[CB][CB + 1];
  __shared__ double Gs[CB][CB + 1];
  const int tid = threadIdx.x;
  const int k0 = j0 + CB * (1 + blockIdx.x);
  for (int t = tid; t < CB * CB; t += 256) {
    const int r = t / CB, c = t - (t / CB) * CB;
    Ss[r][c] = X[(int64_t)(j0 + r) * LB + j0 + c];
    Gs[r][c] = M[(int64_t)(j0 + r) * LB + k0 + c];
  }
  __syncthreads();
  const int a0 = 4 * (tid >> 4), b0 = 4 * (tid & 15);
  double acc[4][4] = {};
  tile_tn(Ss, Gs, a0, b0, acc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) M[(int64_t)(j0 + a0 + i) * LB + k0 + b0 + k] = acc[i][k];
}

// M_KL -= R_JK^T R_JL for J < K <= L; blockIdx.x enumerates the pairs (K, L).
__global__ __launch_bounds__(256) void bc_trail_kernel(double* __restrict__ M, int LB, int j0, int nr) {
  __shared__ double As[CB][CB + 1];
  __shared__ double Bs[CB][CB + 1];
  const int tid = threadIdx.x;
  int idx = blockIdx.x, kb = 0;
  while (idx >= nr - kb) { idx -= nr - kb; ++kb; }
  const int lb = kb + idx;
  const int k0 = j0 + CB * (1 + kb), l0 = j0 + CB * (1 + lb);
  for (int t = tid; t < CB * CB; t += 256) {
    const int r = t / CB, c = t - (t / CB) * CB;
    As[r][c] = M[(int64_t)(j0 + r) * LB + k0 + c];
    Bs[r][c] = M[(int64_t)(j0 + r) * LB + l0 + c];
  }
  __syncthreads();
  const int a0 = 4 * (tid >> 4), b0 = 4 * (tid & 15);
  double acc[4][4] = {};
  tile_tn(As, Bs, a0, b0, acc);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) M[(int64_t)(k0 + a0 + i) * LB + l0 + b0 + k] -= acc[i][k];
}

// X_IJ = -S_II sum_{I < K <= J} R_IK X_KJ for J = I+1+blockIdx.x.
__global__ __launch_bounds__(256) void bc_inv_kernel(const double* __restrict__ M, double* __restrict__ X, int LB,
                                                     int ib) {
  __shared__ double As[CB][CB + 1];
  __shared__ double Bs[CB][CB + 1];
  const int tid = threadIdx.x;
  const int jb = ib + 1 + blockIdx.x;
  const int i0 = ib * CB, jc = jb * CB;
  const int a0 = 4 * (tid >> 4), b0 = 4 * (tid & 15);
  double acc[4][4] = {};
  for (int kb = ib + 1; kb <= jb; ++kb) {
    __syncthreads();
    for (int t = tid; t < CB * CB; t += 256) {
      const int r = t / CB, c = t - (t / CB) * CB;
      As[c][r] = M[(int64_t)(i0 + r) * LB + kb * CB + c];   // As[t][a] = R_IK(a, t)
      Bs[r][c] = X[(int64_t)(kb * CB + r) * LB + jc + c];
    }
    __syncthreads();
    tile_tn(As, Bs, a0, b0, acc);
  }
  __syncthreads();
  for (int t = tid; t < CB * CB; t += 256) {
    const int r = t / CB, c = t - (t / CB) * CB;
    As[c][r] = X[(int64_t)(i0 + r) * LB + i0 + c];   // As[t][a] = S_II(a, t)
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) Bs[a0 + i][b0 + k] = acc[i][k];
  __syncthreads();
  double out[4][4] = {};
  tile_tn(As, Bs, a0, b0, out);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) X[(int64_t)(i0 + a0 + i) * LB + jc + b0 + k] = -out[i][k];
}

// rinv_p[c*LP + k] = R^-1(k, c) for c, k < l; the identity on the padding.
template <typename TQ>
__global__ void bc_rinv_out_kernel(const double* __restrict__ X, int LB, int l, int LP, TQ* __restrict__ rinv_p) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)LP * LP) return;
  const int c = (int)(t / LP), k = (int)(t - (t / LP) * LP);
  double v;
  if (c >= l || k >= l) v = (c == k) ? 1.0 : 0.0;
  else v = (k <= c) ? X[(int64_t)k * LB + c] : 0.0;   // X's blocks below the diagonal are never written
  rinv_p[t] = static_cast<TQ>(v);
}

// r_out (row-major LP x LP) = R, or R R_prev when r_prev is given; identity on the padding.
// One 64 x 64 tile (I <= J) per workgroup.
__global__ __launch_bounds__(256) void bc_r_out_kernel(const double* __restrict__ M, int LB, int l, int LP,
                                                       const double* __restrict__ r_prev, double* __restrict__ r_out,
                                                       int nbk) {
  __shared__ double As[CB][CB + 1];
  __shared__ double Bs[CB][CB + 1];
  const int tid = threadIdx.x;
  int idx = blockIdx.x, ib = 0;
  while (idx >= nbk - ib) { idx -= nbk - ib; ++ib; }
  const int jb = ib + idx;
  const int i0 = ib * CB, j0 = jb * CB;
  const int a0 = 4 * (tid >> 4), b0 = 4 * (tid & 15);
  double acc[4][4] = {};
  if (r_prev) {
    for (int kb = ib; kb <= jb; ++kb) {
      __syncthreads();
      for (int t = tid; t < CB * CB; t += 256) {
        const int r = t / CB, c = t - (t / CB) * CB;
        const int kk = kb * CB + r, jj = j0 + c;
        As[c][r] = M[(int64_t)(i0 + r) * LB + kb * CB + c];
        Bs[r][c] = (kk < l && jj < l) ? r_prev[(int64_t)kk * LP + jj] : 0.0;
      }
      __syncthreads();
      tile_tn(As, Bs, a0, b0, acc);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[i][k] = M[(int64_t)(i0 + a0 + i) * LB + j0 + b0 + k];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = i0 + a0 + i, b = j0 + b0 + k;
      if (a >= LP || b >= LP) continue;
      double v;
      if (a >= l || b >= l) v = (a == b) ? 1.0 : 0.0;
      else v = (b >= a) ? acc[i][k] : 0.0;
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

template <typename TQ>
hipError_t launch_chol_blocked(const double* g, int64_t ldg, int l, int LP, double tau, TQ* rinv_p, double* r_out,
                               const double* r_prev, double* scratch, int* flags, hipStream_t s) {
  const int LB = (LP + CB - 1) / CB * CB;
  const int nbk = LB / CB;
  double* M = scratch;
  double* X = M + (size_t)LB * LB;
  double* gdiag = X + (size_t)LB * LB;
  const int64_t ll = (int64_t)LB * LB;
  hipLaunchKernelGGL(bc_init_kernel, dim3((unsigned)((ll + 255) / 256)), dim3(256), 0, s, g, ldg, l, LB, M, gdiag);
  // X's blocks above the diagonal are all written by the back-substitution; the ones below are never
  // written and never read.
  for (int jb = 0; jb < nbk; ++jb) {
    const int j0 = jb * CB;
    hipLaunchKernelGGL(bc_diag_kernel, dim3(1), dim3(256), 0, s, M, LB, j0, l, gdiag, tau, X, flags);
    const int nr = nbk - 1 - jb;
    if (nr > 0) {
      hipLaunchKernelGGL(bc_panel_kernel, dim3((unsigned)nr), dim3(256), 0, s, M, X, LB, j0);
      hipLaunchKernelGGL(bc_trail_kernel, dim3((unsigned)(nr * (nr + 1) / 2)), dim3(256), 0, s, M, LB, j0, nr);
    }
  }
  for (int ib = nbk - 2; ib >= 0; --ib)
    hipLaunchKernelGGL(bc_inv_kernel, dim3((unsigned)(nbk - 1 - ib)), dim3(256), 0, s, M, X, LB, ib);
  const int64_t lp2 = (int64_t)LP * LP;
  hipLaunchKernelGGL((bc_rinv_out_kernel<TQ>), dim3((unsigned)((lp2 + 255) / 256)), dim3(256), 0, s, X, LB, l, LP,
                     rinv_p);
  if (r_out)
    hipLaunchKernelGGL(bc_r_out_kernel, dim3((unsigned)(nbk * (nbk + 1) / 2)), dim3(256), 0, s, M, LB, l, LP, r_prev,
                       r_out, nbk);
  return hipGetLastError();
}

template hipError_t launch_chol_blocked<float>(const double*, int64_t, int, int, double, float*, double*,
                                               const double*, double*, int*, hipStream_t);
template hipError_t launch_chol_blocked<double>(const double*, int64_t, int, int, double, double*, double*,
                                                const double*, double*, int*, hipStream_t);

// ---------------------------------------------------------------------------
// Block one-sided Jacobi
// ---------------------------------------------------------------------------

__device__ __forceinline__ int bj_player(int pos, int round, int le) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (le - 1);
}

// xs: column p of X at xs[p*ldx + i], i < l.
__global__ void bj_init_kernel(const double* __restrict__ R, int l, int LP, double* __restrict__ xs, int ldx,
                               int ncols) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)ncols * ldx) return;
  const int p = (int)(t / ldx), i = (int)(t - (t / ldx) * ldx);
  xs[t] = (p < l && i < l) ? R[(int64_t)p * LP + i] : 0.0;
}

template <int W>
__global__ __launch_bounds__(512) void bj_round_kernel(double* __restrict__ xs, int ldx, int l, int nbk, int round,
                                                       double tol, int inner_max, int* __restrict__ rot) {
  extern __shared__ double xl[];   // 2W columns, column c at xl[c*l + i]
  constexpr int G = 512 / W;       // lanes per column pair
  constexpr int NI = (W == 16 ? 600 : 1024) / G + 1;   // per-lane slice length bound (l <= 600 resp. 1024)
  __shared__ int any_rot;
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int bI = bj_player(g, round, nbk), bJ = bj_player(nbk - 1 - g, round, nbk);
  auto gcol = [&](int c) { return c < W ? bI * W + c : bJ * W + (c - W); };
  for (int t = tid; t < 2 * W * l; t += 512) {
    const int c = t / l, i = t - (t / l) * l;
    const int gc = gcol(c);
    xl[t] = (gc < l) ? xs[(int64_t)gc * ldx + i] : 0.0;
  }
  const int pi = tid / G, sub = tid - (tid / G) * G;
  int first = 0;
  for (int s = 0; s < inner_max; ++s) {
    __syncthreads();
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int ir = 0; ir < 2 * W - 1; ++ir) {
      const int p = bj_player(pi, ir, 2 * W), q = bj_player(2 * W - 1 - pi, ir, 2 * W);
      if (gcol(p) < l && gcol(q) < l) {   // uniform within the pair group
        double* xp = xl + p * l;
        double* xq = xl + q * l;
        // the lane's slice of both columns, loaded at once (unrolled, predicated) and kept for the rotation
        double av[NI], bv[NI];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
          const int i = sub + u * G;
          av[u] = (i < l) ? xp[i] : 0.0;
          bv[u] = (i < l) ? xq[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NI; ++u) {
          al += av[u] * av[u]; be += bv[u] * bv[u]; ga += av[u] * bv[u];
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, G);
          be += __shfl_xor(be, o, G);
          ga += __shfl_xor(ga, o, G);
        }
        if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double sn = c * t;
#pragma unroll
          for (int u = 0; u < NI; ++u) {
            const int i = sub + u * G;
            if (i < l) {
              xp[i] = c * av[u] - sn * bv[u];
              xq[i] = sn * av[u] + c * bv[u];
            }
          }
          if (sub == 0) any_rot = 1;
        }
      }
      __syncthreads();
    }
    const int r = any_rot;
    if (s == 0) first = r;
    if (!r) break;
  }
  __syncthreads();
  if (tid == 0 && first) atomicAdd(rot, 1);
  for (int t = tid; t < 2 * W * l; t += 512) {
    const int c = t / l, i = t - (t / l) * l;
    const int gc = gcol(c);
    if (gc < l) xs[(int64_t)gc * ldx + i] = xl[t];
  }
}

__global__ void bj_flags_kernel(int* flags, int sweeps, int nonconv) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (nonconv) atomicAdd(&flags[2], 1);
    atomicMax(&flags[3], sweeps);
  }
}

size_t jacobi_blocked_scratch_bytes(int LP) {
  return (size_t)(LP + 32) * LP * sizeof(double) + 64 * sizeof(int);
}

template <typename TU>
hipError_t jacobi_epilogue_launch(const double* xs, int ldx, int l, int LP, double* sigma, double* uhat_d,
                                  TU* uhat_p, TU* vhat_p, hipStream_t s);

template <typename TU>
hipError_t launch_jacobi_blocked(const double* R, int l, int LP, double tol, int max_sweeps, double* sigma,
                                 double* uhat_d, TU* uhat_p, TU* vhat_p, double* scratch, int* flags, hipStream_t s) {
  const int W = (2 * 16 * l * 8 <= 150 * 1024) ? 16 : 8;
  int nbk = (l + W - 1) / W;
  nbk += nbk & 1;
  const int ldx = LP;
  double* xs = scratch;
  int* rot = reinterpret_cast<int*>(scratch + (size_t)(LP + 32) * LP);
  const size_t lds = (size_t)2 * W * l * sizeof(double);
  static bool attr16 = false, attr8 = false;
  if (W == 16 && !attr16) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bj_round_kernel<16>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr16 = true;
  }
  if (W == 8 && !attr8) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&bj_round_kernel<8>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr8 = true;
  }
  const int ncols = nbk * W;
  const int64_t tot = (int64_t)ncols * ldx;
  hipLaunchKernelGGL(bj_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, R, l, LP, xs, ldx, ncols);
  hipError_t e = launch_fill_int(rot, 64, 0, s);
  if (e != hipSuccess) return e;
  const int inner_max = 1;
  int sweep = 0;
  bool converged = (l < 2);
  for (; sweep < max_sweeps && sweep < 64 && !converged; ++sweep) {
    for (int round = 0; round < nbk - 1; ++round) {
      if (W == 16)
        hipLaunchKernelGGL((bj_round_kernel<16>), dim3((unsigned)(nbk / 2)), dim3(512), lds, s, xs, ldx, l, nbk,
                           round, tol, inner_max, rot + sweep);
      else
        hipLaunchKernelGGL((bj_round_kernel<8>), dim3((unsigned)(nbk / 2)), dim3(512), lds, s, xs, ldx, l, nbk,
                           round, tol, inner_max, rot + sweep);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int h = 1;
    e = hipMemcpyAsync(&h, rot + sweep, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    converged = (h == 0);
  }
  hipLaunchKernelGGL(bj_flags_kernel, dim3(1), dim3(64), 0, s, flags, sweep, converged ? 0 : 1);
  return jacobi_epilogue_launch<TU>(xs, ldx, l, LP, sigma, uhat_d, uhat_p, vhat_p, s);
}

template hipError_t launch_jacobi_blocked<float>(const double*, int, int, double, int, double*, double*, float*,
                                                 float*, double*, int*, hipStream_t);
template hipError_t launch_jacobi_blocked<double>(const double*, int, int, double, int, double*, double*, double*,
                                                  double*, double*, int*, hipStream_t);

}  // namespace rsvd
