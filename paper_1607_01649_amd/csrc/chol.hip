// Cholesky factorisation of the l x l Gram matrix of CholeskyQR, in FP64, in
// one workgroup.
//
// orth(Y) (Section 2.3: any unpivoted orthonormalisation will do) is computed
// as CholeskyQR: G = Y^T Y = R^T R, Q = Y R^-1.  This kernel factors G and at
// the same time builds R^-T (the elimination applied to an identity block), so
// the triangular apply that follows is a plain panel product with R^-1.
//
// l <= 128: right-looking block Cholesky over 16 x 16 blocks held in LDS.  The
// diagonal blocks are factored by one wave in registers (unscaled elimination,
// pivot d_j = U(j, j), R = D^-1/2 U, R^-T = D^-1/2 T); the block row solve,
// the trailing update and the carried inverse run on the FP64 MFMA.  Larger l
// goes to the blocked multi-workgroup form in blocked.hip.
//
// Numerically dependent columns (pivot <= tau_rel * G_jj) are dropped: they
// take no part in later eliminations, row j of R and column j of R^-1 come out
// zero (so column j of Q is exactly zero).  Counted in flags[1]; a non-finite
// pivot is counted in flags[0].
#include <algorithm>

#include "internal.hpp"

namespace rsvd {

constexpr int kCholThreads = 512;   // eight waves
constexpr int kCholWaves = kCholThreads / 64;
constexpr int kCholB = 16;          // block size (one FP64 MFMA tile)
constexpr int kWdPitch = 17;        // LDS pitch of a diagonal block of W (odd: conflict-free column reads)

// 1/x for finite x > 0: hardware estimate and two Newton steps.
__device__ __forceinline__ double chol_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Value of lane X of the caller's 16-lane row (64-bit DPP move with row_newbcast, gfx90a and later).
template <int X>
__device__ __forceinline__ double row_lane_f64(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + X, 0xF, 0xF, false);
}

// u[X] = lane X's value of w, for X = X0 .. 15.
template <int X0, int X>
__device__ __forceinline__ void row_gather(double (&u)[16], double w) {
  if constexpr (X < 16) {
    u[X] = row_lane_f64<X>(w);
    row_gather<X0, X + 1>(u, w);
  }
}

// Factorisation of one 16 x 16 diagonal block by one wave, in registers.  Every 16-lane row holds the
// block (the four rows compute the same): lane c holds column c of the symmetric block, v[x] = A(x, c),
// and column c of T, t[x] (the identity at the start).  Unscaled elimination with pivot d_j = A(j, j):
//     A(x, c) -= A(x, j) A(j, c) / d_j      (x > j, c > j)
//     T(x, c) -= A(x, j) T(j, c) / d_j      (x > j)
// A(j, c) and T(j, c) are the lane's own entries; A(x, j) = A(j, x) (the trailing block stays symmetric)
// is lane x's entry j, taken by a row broadcast, as is the pivot; the loops over x start past j at
// compile time.  R = D^-1/2 U and R^-T = D^-1/2 T.  A pivot takes part only when d_j > tau_rel G_jj and
// d_j > 0 with j < nv (a NaN fails the test); otherwise 1/d_j is taken as 0, so that its row of R and its
// row and column of R^-T come out zero.  Lane j keeps d_j and 1/d_j (dj, dl).
template <int J>
__device__ __forceinline__ void chol_pivot(double (&v)[16], double (&t)[16], double& dj, double& dl, double tg,
                                           int nv, int c) {
  const double d = row_lane_f64<J>(v[J]);
  const double thr = row_lane_f64<J>(tg);   // tau_rel G_jj
  double u[16];
  row_gather<J + 1, J + 1>(u, v[J]);
  const bool keep = (J < nv) & (d > thr) & (d > 0.0) & (d < 1.79769313486231570815e308);
  const double dinv = keep ? chol_rcp(d) : 0.0;
  const double f = (c <= J) ? 0.0 : v[J] * dinv;
  const double ft = t[J] * dinv;
#pragma unroll
  for (int x = J + 1; x < 16; ++x) {
    v[x] -= u[x] * f;
    t[x] -= u[x] * ft;
    asm volatile("" : "+v"(t[x]));   // update T now: deferring it keeps every broadcast value live
  }
  dj = (c == J) ? d : dj;
  dl = (c == J) ? dinv : dl;
}

template <int J>
__device__ __forceinline__ void chol_pivots(double (&v)[16], double (&t)[16], double& dj, double& dl, double tg,
                                            int nv, int c) {
  if constexpr (J < kCholB) {
    chol_pivot<J>(v, t, dj, dl, tg, nv, c);
    chol_pivots<J + 1>(v, t, dj, dl, tg, nv, c);
  }
}

// Row scale of R and R^-T: out[x] = lane x's value of r.
template <int X>
__device__ __forceinline__ void row_all(double (&out)[16], double r) {
  if constexpr (X < 16) {
    out[X] = row_lane_f64<X>(r);
    row_all<X + 1>(out, r);
  }
}

// Diagonal block at blk (leading dimension ldb, the symmetric block in both triangles) -> R_JJ into blk
// (zero below the diagonal) and W_JJ = R_JJ^-T into wblk (pitch kWdPitch, zero above the diagonal).
// gd: the original diagonal entries of the block's columns.  One wave.  Pivots past nv (padding) are not
// counted; a valid pivot that does not take part is counted as dropped (flags[1]) or, when d_j or G_jj
// is not finite, as non-finite (flags[0]).
__device__ __forceinline__ void chol_block(double* __restrict__ blk, int ldb, const double* __restrict__ gd, int nv,
                                           double tau_rel, int lane, double* __restrict__ wblk, int& bad,
                                           int& dropped) {
  const int c = lane & 15;
  double v[16], t[16];
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    v[x] = blk[x * ldb + c];
    t[x] = (x == c) ? 1.0 : 0.0;
  }
  const double g0 = gd[c];
  double dj = 0.0, dl = 0.0;
  chol_pivots<0>(v, t, dj, dl, tau_rel * g0, nv, c);
  const bool valid = c < nv && lane < 16;
  const bool nonfinite = valid && !(fabs(dj) <= 1.79769313486231570815e308 && fabs(g0) <= 1.79769313486231570815e308);
  const bool drop = valid && !nonfinite && dl == 0.0;
  bad += __builtin_popcountll(__ballot(nonfinite));
  dropped += __builtin_popcountll(__ballot(drop));
  double rs[16];
  row_all<0>(rs, dl > 0.0 ? sqrt(dl) : 0.0);
  if (lane < 16) {
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      blk[x * ldb + c] = (c >= x) ? v[x] * rs[x] : 0.0;
      wblk[x * kWdPitch + c] = (c <= x) ? t[x] * rs[x] : 0.0;
    }
  }
}

// One 16 x 16 FP64 MFMA product D = C + sum_k A(i, k) B(k, j) over k < 16, with lane (g, i) supplying
// A(i, 4 s + g) and B(4 s + g, i) at step s; element e of lane (g, j) of the result is D(g + 4 e, j).
__device__ __forceinline__ f64x4 mma16(const double* __restrict__ A, int sai, int sak, const double* __restrict__ B,
                                       int sbk, int sbj, f64x4 acc, int lane, double sign) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + g;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * A[i * sai + k * sak], B[k * sbk + i * sbj], acc, 0, 0, 0);
  }
  return acc;
}

// The block elimination on an LP x LP matrix held in LDS (M with pitch MP, nb = LP / 16 blocks; on entry the
// blocks on and above the block diagonal hold the symmetric matrix, both triangles of the diagonal blocks,
// and the blocks below are zero; Wd holds nb diagonal blocks of pitch kWdPitch).  On exit the upper blocks
// hold R, the diagonal blocks of R^-T are in Wd and its blocks below the diagonal in M.  gd: the original
// diagonal entries (the drop rule's reference), nvalid: the columns that take part (the rest is padding).
// All eight waves of the workgroup call it.
__device__ __forceinline__ void chol_lds_factor(double* __restrict__ M, int MP, double* __restrict__ Wd, int nb,
                                                int nvalid, const double* __restrict__ gd, double tau_rel,
                                                int& bad, int& dropped) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lg = lane >> 4, lc = lane & 15;
  // Iteration J (from -1): T(J) -- the trailing update by block row J (none for J = -1) by waves 1..3 and,
  // by wave 0, the update and factorisation of diagonal block J+1 -- then P(J+1).
  for (int J = -1; J < nb - 1; ++J) {
    const int r0 = kCholB * J, r1 = r0 + kCholB;
    const double* WJ = Wd + (J < 0 ? 0 : J) * kCholB * kWdPitch;
    if (wv == 0) {
      double* dblk = M + r1 * MP + r1;
      if (J >= 0) {
        const double* rk = M + r0 * MP + r1;   // R_{J, J+1}
        f64x4 acc;
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = dblk[(lg + 4 * e) * MP + lc];
        acc = mma16(rk, 1, MP, rk, MP, 1, acc, lane, -1.0);
#pragma unroll
        for (int e = 0; e < 4; ++e) dblk[(lg + 4 * e) * MP + lc] = acc[e];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      chol_block(dblk, MP, gd + r1, nvalid - r1, tau_rel, lane, Wd + (J + 1) * kCholB * kWdPitch, bad, dropped);
    } else if (J >= 0) {
      const int nt = nb - 1 - J;                    // block rows below J
      const int nupper = nt * (nt + 1) / 2 - 1;     // trailing A blocks except (J+1, J+1)
      const int ntask = nupper + nt * (J + 1);
      for (int task = wv - 1; task < ntask; task += kCholWaves - 1) {
        int K, L;
        const double* bop;
        int sbk;
        if (task < nupper) {
          // upper blocks (K, L), J < K <= L, in row order, (J+1, J+1) skipped
          int t = task + 1, k = 0;
          while (t >= nt - k) { t -= nt - k; ++k; }
          K = J + 1 + k;
          L = K + t;
          bop = M + r0 * MP + kCholB * L;
          sbk = MP;
        } else {
          const int t = task - nupper;
          K = J + 1 + t / (J + 1);
          L = t - (t / (J + 1)) * (J + 1);          // M <= J
          bop = (L == J) ? WJ : M + r0 * MP + kCholB * L;
          sbk = (L == J) ? kWdPitch : MP;
        }
        double* cblk = M + kCholB * K * MP + kCholB * L;
        const double* rk = M + r0 * MP + kCholB * K;   // R_JK
        f64x4 acc;
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = cblk[(lg + 4 * e) * MP + lc];
        acc = mma16(rk, 1, MP, bop, sbk, 1, acc, lane, -1.0);
#pragma unroll
        for (int e = 0; e < 4; ++e) cblk[(lg + 4 * e) * MP + lc] = acc[e];
      }
    }
    __syncthreads();
    // P(J+1): block row J+1 of R (right of the diagonal) and of W (left of it)
    const int Jn = J + 1;
    const double* WJn = Wd + Jn * kCholB * kWdPitch;
    for (int task = wv; task < nb - 1; task += kCholWaves) {
      const int col = task < Jn ? task : task + 1;   // the block column, Jn skipped
      double* blk = M + r1 * MP + kCholB * col;
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
      acc = mma16(WJn, kWdPitch, 1, blk, MP, 1, acc, lane, 1.0);
#pragma unroll
      for (int e = 0; e < 4; ++e) blk[(lg + 4 * e) * MP + lc] = acc[e];
    }
    __syncthreads();
  }
}

// l <= 128: one workgroup of eight waves, G in LDS as an LP x (LP + 1) matrix M of 16 x 16 blocks.  The
// blocks on and above the diagonal hold A (the trailing matrix) and become R; the blocks below it hold T
// (the accumulated elimination of the identity) and become R^-T, whose diagonal blocks live apart in Wd.
// Right-looking block Cholesky with the inverse carried along (block forward substitution of R^T X = I):
//   block column J, with R_JJ and W_JJ = R_JJ^-T from the factorisation of the diagonal block:
//     P(J): R_JK = W_JJ A_JK (K > J) and W_JM = W_JJ T_JM (M < J)            [one MFMA task per wave]
//     T(J): A_KL -= R_JK^T R_JL (J < K <= L), T_KM -= R_JK^T W_JM (K > J, M <= J); wave 0 first updates
//           block (J+1, J+1) and factors it, in registers, while the others take the remaining blocks.
// Two barriers per block column.  The elimination is the pivot-by-pivot one regrouped by blocks, with the
// same drop rule (against the original diagonal) and the same unscaled pivots inside each block.
template <typename TQ>
__global__ __launch_bounds__(kCholThreads) void chol_blk_kernel(const double* __restrict__ g, int64_t ldg, int l,
                                                                 int LP, double tau_rel, TQ* __restrict__ rinv_p,
                                                                 double* __restrict__ r_out,
                                                                 const double* __restrict__ r_prev,
                                                                 int* __restrict__ flags,
                                                                 const int* __restrict__ skip_in,
                                                                 int* __restrict__ skip_out, double kappa2_max) {
  extern __shared__ __align__(16) double chol_lds[];
  if (skip_in && *skip_in) {   // a skipped second CholeskyQR pass: R^-1 = I (uniform: every thread reads the flag)
    for (int e = threadIdx.x; e < LP * LP; e += kCholThreads)
      rinv_p[e] = static_cast<TQ>((e / LP) == (e - (e / LP) * LP) ? 1.0 : 0.0);
    return;
  }
  const int MP = LP + 1;
  const int nb = LP / kCholB;
  double* M = chol_lds;                    // LP x MP
  double* Wd = chol_lds + LP * MP;         // nb blocks of 16 x kWdPitch
  __shared__ double gdiag[128];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lg = lane >> 4, lc = lane & 15;

  // load: A blocks (on and above the block diagonal) from G (symmetric, both triangles stored); T blocks
  // (below) zero.  A thread takes four consecutive rows a .. a+3 of column b (one block), loaded before
  // any store.
  {
    const int ng = LP / 4;                       // row quads per column
    const int nitem = LP * ng;
    constexpr int kIt = 128 * 32 / kCholThreads;  // items per thread at LP = 128
    double gv[kIt][4];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int item = tid + kCholThreads * it;
      const int b = item / ng, a = 4 * (item - (item / ng) * ng);
      const bool up = item < nitem && b < l && (a >> 4) <= (b >> 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) gv[it][e] = (up && a + e < l) ? g[(int64_t)b * ldg + a + e] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int item = tid + kCholThreads * it;
      if (item >= nitem) continue;
      const int b = item / ng, a = 4 * (item - (item / ng) * ng);
#pragma unroll
      for (int e = 0; e < 4; ++e) M[(a + e) * MP + b] = gv[it][e];
      if ((b & ~3) == a) {
        const int e = b & 3;
        gdiag[b] = e == 0 ? gv[it][0] : e == 1 ? gv[it][1] : e == 2 ? gv[it][2] : gv[it][3];
      }
    }
  }
  __syncthreads();
  int bad = 0, dropped = 0;
  chol_lds_factor(M, MP, Wd, nb, l, gdiag, tau_rel, bad, dropped);
  if (wv == 0 && lane == 0) {
    if (bad) atomicAdd(&flags[0], bad);
    if (dropped) atomicAdd(&flags[1], dropped);
  }
  if (skip_out) {
    // Condition bound of the panel X with columns scaled to unit norm (S = diag(G_jj)^-1/2): kappa_2(X S) <=
    // ||R S||_F ||S^-1 R^-1||_F, with ||R S||_F^2 = l (column j of R has squared norm G_jj) and
    // ||S^-1 R^-1||_F^2 = sum_i G_ii ||column i of R^-T||^2.  One pass of CholeskyQR then leaves X R^-1
    // orthonormal to about kappa^2 u (the FP64 Gram) plus kappa times the panel's rounding.
    // Every entry (i, c), c >= i, of R^-1 by its own thread (about a dozen independent LDS reads each).
    __shared__ double kpart[kCholWaves];
    double f = 0.0;
    for (int e = tid; e < l * l; e += kCholThreads) {
      const int i = e / l, c = e - (e / l) * l;
      if (c >= i) {
        const int bi = i >> 4;
        const double v = (c >> 4) == bi ? Wd[bi * kCholB * kWdPitch + (c & 15) * kWdPitch + (i & 15)] : M[c * MP + i];
        f = fma(gdiag[i] * v, v, f);
      }
    }
    f = wave_sum(f);
    if (lane == 0) kpart[wv] = f;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < kCholWaves; ++w) t += kpart[w];
      *skip_out = (bad == 0 && dropped == 0 && (double)l * t <= kappa2_max) ? 1 : 0;
    }
  }
  // R^-1 in panel layout: rinv_p[c*LP + k] = R^-T(c, k); identity on padding.  A thread writes four
  // consecutive entries (one block).
  const int ng = LP / 4;
  for (int item = tid; item < LP * ng; item += kCholThreads) {
    const int cc = item / ng, k0 = 4 * (item - (item / ng) * ng);
    const int bc = cc >> 4, bk = k0 >> 4;
    double v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = k0 + e;
      if (cc >= l || kk >= l) v[e] = (cc == kk) ? 1.0 : 0.0;
      else if (bc == bk) v[e] = Wd[bc * kCholB * kWdPitch + (cc & 15) * kWdPitch + (kk & 15)];
      else v[e] = (bk < bc) ? M[cc * MP + kk] : 0.0;
    }
    TQ* o = rinv_p + (int64_t)cc * LP + k0;
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = static_cast<TQ>(v[e]);
  }
  if (!r_out) return;
  if (!r_prev) {
    for (int item = tid; item < LP * ng; item += kCholThreads) {
      const int x = item / ng, y0 = 4 * (item - (item / ng) * ng);
      double* o = r_out + (int64_t)x * LP + y0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int y = y0 + e;
        double v;
        if (x >= l || y >= l) v = (x == y) ? 1.0 : 0.0;
        else v = ((x >> 4) <= (y >> 4)) ? M[x * MP + y] : 0.0;
        o[e] = v;
      }
    }
    return;
  }
  // R R_prev (the product of the two passes of CholeskyQR2), block (I, Jb) for I <= Jb: the sum over
  // I <= K <= Jb of R_IK R_prev_KJb (both upper triangular; R_prev has identity padding).
  const int nblk = nb * (nb + 1) / 2;
  for (int task = wv; task < nblk; task += kCholWaves) {
    int t = task, I = 0;
    while (t >= nb - I) { t -= nb - I; ++I; }
    const int Jb = I + t;
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int K = I; K <= Jb; ++K)
      acc = mma16(M + kCholB * I * MP + kCholB * K, MP, 1, r_prev + (int64_t)kCholB * K * LP + kCholB * Jb, LP, 1,
                  acc, lane, 1.0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int x = kCholB * I + lg + 4 * e, y = kCholB * Jb + lc;
      r_out[(int64_t)x * LP + y] = (x >= l || y >= l) ? ((x == y) ? 1.0 : 0.0) : acc[e];
    }
  }
  for (int task = wv; task < nb * nb; task += kCholWaves) {   // blocks below the diagonal
    const int I = task / nb, Jb = task - (task / nb) * nb;
    if (I <= Jb) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int x = kCholB * I + lg + 4 * e, y = kCholB * Jb + lc;
      r_out[(int64_t)x * LP + y] = 0.0;
    }
  }
}

// Diagonal block J of the blocked form (l > 128): rows and columns j0 .. j0+63 of its working matrix Mg
// (row-major, leading dimension LB; the entries on and above the block's diagonal are current) factored
// by the same block elimination as the one-workgroup kernel: R_JJ into Mg's block (zero below its
// diagonal) and S_JJ = R_JJ^-1 into X's diagonal block (row-major, zero below the diagonal).  gdiag: the
// original diagonal of G (the drop rule's reference); columns past l are padding.
__global__ __launch_bounds__(kCholThreads) void chol_diag64_kernel(double* __restrict__ Mg, int LB, int j0, int l,
                                                                 const double* __restrict__ gdiag, double tau_rel,
                                                                 double* __restrict__ X, int* __restrict__ flags,
                                                                 const int* __restrict__ skip) {
  if (skip && *skip) return;   // a skipped second CholeskyQR pass
  constexpr int D = 64, MP = D + 1, nb = D / kCholB;
  __shared__ __align__(16) double M[D * MP];
  __shared__ __align__(16) double Wd[nb * kCholB * kWdPitch];
  const int tid = threadIdx.x;
  const int nv = min(D, l - j0);
  // the symmetric block in both triangles of the diagonal 16 x 16 blocks and above them; zero below
  for (int e = tid; e < D * D; e += kCholThreads) {
    const int a = e / D, b = e - (e / D) * D;
    double v = 0.0;
    if ((a >> 4) <= (b >> 4) && a < nv && b < nv) {
      const int r = min(a, b), c = max(a, b);
      v = Mg[(int64_t)(j0 + r) * LB + j0 + c];
    }
    M[a * MP + b] = v;
  }
  __syncthreads();
  int bad = 0, dropped = 0;
  chol_lds_factor(M, MP, Wd, nb, nv, gdiag + j0, tau_rel, bad, dropped);
  if (tid == 0) {
    if (bad) atomicAdd(&flags[0], bad);
    if (dropped) atomicAdd(&flags[1], dropped);
  }
  for (int e = tid; e < D * D; e += kCholThreads) {
    const int a = e / D, b = e - (e / D) * D;
    double sv = 0.0;   // S_JJ(a, b) = R^-T(b, a)
    if (a <= b)
      sv = ((a >> 4) == (b >> 4)) ? Wd[(a >> 4) * kCholB * kWdPitch + (b & 15) * kWdPitch + (a & 15)] : M[b * MP + a];
    Mg[(int64_t)(j0 + a) * LB + j0 + b] = (a <= b) ? M[a * MP + b] : 0.0;
    X[(int64_t)(j0 + a) * LB + j0 + b] = sv;
  }
}

hipError_t launch_chol_diag64(double* M, int LB, int j0, int l, const double* gdiag, double tau_rel, double* X,
                              int* flags, hipStream_t s, const int* skip) {
  if (j0 < 0 || j0 >= l || LB % 64 != 0 || j0 + 64 > LB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_diag64_kernel, dim3(1), dim3(kCholThreads), 0, s, M, LB, j0, l, gdiag, tau_rel, X, flags,
                     skip);
  return hipGetLastError();
}

template <typename TQ>
hipError_t launch_chol(const double* g, int64_t ldg, int l, int LP, double tau_rel, TQ* rinv_p, double* r_out,
                       const double* r_prev, double* scratch, int* flags, hipStream_t s, int* skip_out,
                       double kappa_max, const int* skip_in) {
  if (l < 1 || l > 1024) return hipErrorInvalidValue;
  if (skip_in && r_out) return hipErrorInvalidValue;   // a skippable pass only writes R^-1
  if (LP <= 128) {
    if (LP % kCholB != 0) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_blk_kernel<TQ>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (128 * 129 + 8 * kCholB * kWdPitch) * (int)sizeof(double));
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    const size_t sh = ((size_t)LP * (LP + 1) + (size_t)(LP / kCholB) * kCholB * kWdPitch) * sizeof(double);
    hipLaunchKernelGGL((chol_blk_kernel<TQ>), dim3(1), dim3(kCholThreads), sh, s, g, ldg, l, LP, tau_rel, rinv_p,
                       r_out, r_prev, flags, skip_in, skip_out, kappa_max * kappa_max);
  } else {
    if (!scratch) return hipErrorInvalidValue;
    return launch_chol_blocked<TQ>(g, ldg, l, LP, tau_rel, rinv_p, r_out, r_prev, scratch, flags, s, skip_out,
                                   kappa_max * kappa_max, skip_in);
  }
  return hipGetLastError();
}

template hipError_t launch_chol<float>(const double*, int64_t, int, int, double, float*, double*, const double*,
                                       double*, int*, hipStream_t, int*, double, const int*);
template hipError_t launch_chol<double>(const double*, int64_t, int, int, double, double*, double*, const double*,
                                        double*, int*, hipStream_t, int*, double, const int*);

}  // namespace rsvd
