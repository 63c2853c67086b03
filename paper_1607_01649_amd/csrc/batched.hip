// Batched, tolerance-driven compression of many small blocks in one
// persistent launch.
//
// Each workgroup (512 threads) takes blocks from an atomic queue (largest
// first) and compresses one block K (m_b x n_b <= 512 x 512, FP32 row-major)
// to the relative tolerance eps with the given-tolerance scheme of Sections
// 12-14:
//   Q = orth(K Omega) with l0 = 16 Gaussian columns, B = Q^T K;
//   certificate (Section 14, 10 probes, alpha = 1/10) of the pair (Q, B):
//     bound = 10 sqrt(2/pi) max_i ||(K - Q B) g_i||;
//   while bound > eps sigma_hat_1 / 2: b = 8 more Gaussian columns (Omega's
//   continuation), projected against Q twice, orthonormalised and appended
//   together with their rows of B (Figure 12 with the residual applied
//   implicitly); the probe residual is updated incrementally;
//   SVD of B via the eigen-decomposition of B B^T (cyclic Jacobi, FP64), kept
//   singular values > eps sigma_hat_1 / 2, U = Q U_hat, V = B^T U_hat S^-1.
// All accumulation is FP64 (the probe threshold sits near FP32's noise floor
// at eps = 1e-6).  Thread t owns row t of the row-indexed quantities (Y, Q,
// E) and column t of the column-indexed ones (B^T); cross-thread sums go
// through 64-row chunks staged in LDS.
//
// Per-block random streams: 16*blk + 4 (Omega and its continuation),
// 16*blk + 6 (probes), same Philox4x32-10 / Box-Muller mapping as the
// single-matrix path.
#include "internal.hpp"

namespace rsvd {

constexpr int BT = 512;       // threads per workgroup (one block row / column each)
constexpr int BROWS = 512;    // max rows / columns of a block
constexpr int RMAX = 64;      // max basis width
constexpr int L0 = 16;        // initial sketch width
constexpr int BG = 8;         // growth block
constexpr int NP = 10;        // certificate probes
constexpr int CH = 64;        // rows per LDS chunk of the cross-thread sums
constexpr int KC = 16;        // columns of K per staged tile in the row-owned products
constexpr int KLD = KC + 1;   // LDS pitch of a staged K row

struct BatchedArgs {
  int nblk;
  const int* m;
  const int* n;
  const float* const* A;
  const int* lda;
  double eps;
  int rank_cap;       // <= RMAX
  uint64_t seed;
  float* U;
  double* S;
  float* V;
  const int64_t* offU;
  const int64_t* offV;
  int* rank;
  int* status;
  const int* order;   // processing order (largest first)
  int* queue;         // work counter, zero before launch
  double* scratch;    // per-workgroup scratch
  int64_t scratch_per_wg;
};

// Philox4x32-10, same as rng.hip (kept local so this file stands alone).
__device__ __forceinline__ void bphilox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
    uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// Rows 2*i2 and 2*i2+1 of column `col` of the Gaussian family (seed, stream).
__device__ __forceinline__ void bgauss_pair(uint64_t seed, uint32_t stream, uint32_t i2, uint32_t col, double& z0,
                                            double& z1) {
  uint32_t c[4] = {i2, col, stream, 0u};
  bphilox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  uint64_t v1 = ((((uint64_t)c[0]) << 32) | c[1]) >> 11;
  uint64_t v2 = ((((uint64_t)c[2]) << 32) | c[3]) >> 11;
  const double s53 = 1.1102230246251565404e-16;
  double u1 = ((double)v1 + 0.5) * s53, u2 = ((double)v2 + 0.5) * s53;
  double rad = sqrt(-2.0 * log(u1)), th = 6.283185307179586477 * u2;
  z0 = rad * cos(th);
  z1 = rad * sin(th);
}

// Stage rows [j0, j0+KC) of `nc` Gaussian columns into lds[jj*ldl + c] (zero past n):
// columns [0, nc0) from stream s0 starting at column col0, columns [nc0, nc) from stream s1.
__device__ void stage_gauss(double* lds, int ldl, int j0, int n, int nc, int nc0, uint64_t seed, uint32_t s0,
                            int col0, uint32_t s1) {
  const int pairs = KC / 2;
  for (int t = threadIdx.x; t < pairs * nc; t += BT) {
    int c = t / pairs, i2 = t - (t / pairs) * pairs;
    int j = j0 + 2 * i2;
    double z0 = 0.0, z1 = 0.0;
    if (j < n) {
      if (c < nc0) bgauss_pair(seed, s0, (uint32_t)(j >> 1), (uint32_t)(col0 + c), z0, z1);
      else bgauss_pair(seed, s1, (uint32_t)(j >> 1), (uint32_t)(c - nc0), z0, z1);
    }
    lds[(2 * i2) * ldl + c] = z0;
    lds[(2 * i2 + 1) * ldl + c] = (j + 1 < n) ? z1 : 0.0;
  }
}

// Stage columns [j0, j0+KC) of rows [0, m) of K into tile[r*KLD + c] (zero past n).  Each
// group of KC threads reads KC consecutive floats of one row, so the global reads are
// contiguous; the odd LDS row pitch keeps the row-per-thread reads conflict-free.
__device__ void stage_k(const float* __restrict__ A, int lda, int m, int n, int j0, float* tile) {
  for (int t = threadIdx.x; t < m * KC; t += BT) {
    const int r = t / KC, c = t - (t / KC) * KC;
    tile[r * KLD + c] = (j0 + c < n) ? A[(int64_t)r * lda + j0 + c] : 0.0f;
  }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < BT / 64; ++w) t += red[w];
  return t;
}

// C[a*ldc + b] = sum over rows of X[row][a] * Z[row][b] for a < na, b < nbz, where row
// i's vectors are held by thread i in xr, zr.
template <int NX, int NZ>
__device__ void rows_inner(const double (&xr)[NX], int na, const double (&zr)[NZ], int nbz, int rows, double* stage,
                           double* C, int ldc) {
  double acc = 0.0;
  const int nout = na * nbz;
  const int o = threadIdx.x;
  const int a = o / max(nbz, 1), b = o - a * max(nbz, 1);
  for (int r0 = 0; r0 < rows; r0 += CH) {
    __syncthreads();
    if (threadIdx.x >= r0 && threadIdx.x < r0 + CH) {
      const int rr = threadIdx.x - r0;
      const bool ok = threadIdx.x < rows;
#pragma unroll
      for (int q = 0; q < NX; ++q) stage[rr * (NX + NZ) + q] = ok ? xr[q] : 0.0;
#pragma unroll
      for (int q = 0; q < NZ; ++q) stage[rr * (NX + NZ) + NX + q] = ok ? zr[q] : 0.0;
    }
    __syncthreads();
    if (o < nout) {
      double sacc = 0.0;
      for (int rr = 0; rr < CH; ++rr) sacc += stage[rr * (NX + NZ) + a] * stage[rr * (NX + NZ) + NX + b];
      acc += sacc;
    }
  }
  __syncthreads();
  if (o < nout) C[a * ldc + b] = acc;
  __syncthreads();
}

// In-LDS Cholesky of the NC x NC Gram G (row-major, ld NC <= 16) and the upper-triangular
// R^-1 (row-major, ld 16) written to Ri; columns with a pivot <= tau * G_jj are dropped
// (zero column of R^-1).  All threads take part (thread a*NC + b owns entry (a, b)); same
// unscaled elimination as the single-matrix Cholesky: U(a, b) -= f_a U(j, b) for b >= a,
// T(a, b) -= f_a T(j, b), f_a = U(j, a) / d_j.  Tm: NC*NC doubles of LDS scratch.
template <int NC>
__device__ void small_chol_inv(double* G, double* Tm, double* Ri, double tau) {
  __shared__ double gd[16], rs[16];
  const int tid = threadIdx.x;
  const int a = tid / NC, b = tid - (tid / NC) * NC;
  const bool own = tid < NC * NC;
  if (own) Tm[tid] = (a == b) ? 1.0 : 0.0;
  if (tid < NC) gd[tid] = G[tid * NC + tid];
  __syncthreads();
  for (int j = 0; j < NC; ++j) {
    const double d = G[j * NC + j];
    const bool drop = !(d > tau * gd[j]) || !isfinite(d);
    if (own && !drop && a > j) {
      const double f = G[j * NC + a] / d;
      if (b >= a) G[a * NC + b] -= f * G[j * NC + b];
      Tm[a * NC + b] -= f * Tm[j * NC + b];
    }
    if (tid == 0) rs[j] = drop ? 0.0 : 1.0 / sqrt(d);
    __syncthreads();
  }
  // R^-1(k, c) = R^-T(c, k) = T(c, k) / sqrt(d_c)
  if (tid < 256) {
    const int k = tid / 16, c = tid % 16;
    Ri[tid] = (c < NC && k < NC && k <= c) ? Tm[c * NC + k] * rs[c] : 0.0;
  }
  __syncthreads();
}

// Eigen-decomposition of the symmetric positive semi-definite nc x nc matrix M (LDS, ld
// RMAX, nc <= RMAX) by two-sided Jacobi with the parallel round-robin ordering: with
// N = nc rounded up to even (a zero dummy row and column when nc is odd), each of the N-1
// rounds of a sweep rotates N/2 disjoint pairs at once, so one round is one update
// M <- J^T M J, V <- V J by all threads.  Pairs of round r (circle method): player N-1
// meets r, and (r + i) mod (N-1) meets (r - i) mod (N-1) for i = 1 .. N/2-1.  A pair is
// skipped when its off-diagonal entry is negligible relative to its own diagonal (1e-15)
// or to the largest diagonal entry (1e-16: below that it is rounding noise of M); the
// sweeps end when one passes without a rotation (at most 30).  Eigenvectors in Vm (ld
// RMAX); eigenvalues on the diagonal of M.  All threads call it; it ends with a sync.
__device__ void small_eig(double* M, double* Vm, int nc) {
  __shared__ double cf[RMAX], df[RMAX], nd[RMAX];
  __shared__ int prt[RMAX], rot[RMAX];
  __shared__ int any_rot;
  __shared__ double dmax_s;
  constexpr int PER = RMAX * RMAX / BT;
  const int tid = threadIdx.x;
  const int N = (nc + 1) & ~1;
  for (int t = tid; t < N * N; t += BT) {
    const int a = t / N, b = t - (t / N) * N;
    Vm[a * RMAX + b] = (a == b) ? 1.0 : 0.0;
    if (a == nc || b == nc) M[a * RMAX + b] = 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (tid == 0) {
      double d = 0.0;
      for (int a = 0; a < nc; ++a) d = fmax(d, M[a * RMAX + a]);
      dmax_s = d;
      any_rot = 0;
    }
    __syncthreads();
    const double dmax = dmax_s;
    for (int r = 0; r < N - 1; ++r) {
      if (tid < N / 2) {
        int p = (tid == 0) ? N - 1 : (r + tid) % (N - 1);
        int q = (r - tid + (N - 1)) % (N - 1);
        if (p > q) { const int x = p; p = q; q = x; }
        const double apq = M[p * RMAX + q], app = M[p * RMAX + p], aqq = M[q * RMAX + q];
        double c = 1.0, sn = 0.0, tapq = 0.0;
        const bool go = !(fabs(apq) <= 1e-15 * sqrt(fabs(app * aqq)) || fabs(apq) <= 1e-16 * dmax);
        if (go) {
          const double th = (aqq - app) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sn = t * c;
          tapq = t * apq;
          any_rot = 1;
        }
        prt[p] = q; prt[q] = p;
        cf[p] = c; df[p] = -sn;
        cf[q] = c; df[q] = sn;
        nd[p] = app - tapq; nd[q] = aqq + tapq;
        rot[p] = go; rot[q] = go;
      }
      __syncthreads();
      double mv[PER], vv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int t = tid + u * BT;
        mv[u] = 0.0;
        vv[u] = 0.0;
        if (t < N * N) {
          const int x = t / N, y = t - (t / N) * N;
          const int px = prt[x], py = prt[y];
          const double cx = cf[x], dx = df[x], cy = cf[y], dy = df[y];
          if (x == y) mv[u] = nd[x];
          else if (py == x && rot[x]) mv[u] = 0.0;
          else
            mv[u] = cx * (cy * M[x * RMAX + y] + dy * M[x * RMAX + py]) +
                    dx * (cy * M[px * RMAX + y] + dy * M[px * RMAX + py]);
          vv[u] = cy * Vm[x * RMAX + y] + dy * Vm[x * RMAX + py];
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int t = tid + u * BT;
        if (t < N * N) {
          const int x = t / N, y = t - (t / N) * N;
          M[x * RMAX + y] = mv[u];
          Vm[x * RMAX + y] = vv[u];
        }
      }
      __syncthreads();
    }
    if (!any_rot) break;
    __syncthreads();
  }
}

__global__ __launch_bounds__(BT) void batched_kernel(BatchedArgs g) {
  __shared__ double lds[2 * RMAX * RMAX];   // phase-dependent union (64 KB)
  __shared__ double H[RMAX * NP];
  __shared__ double Ri[16 * 16];
  __shared__ double red[BT / 64];
  __shared__ double sig[RMAX];
  __shared__ double sgn[RMAX];
  __shared__ int perm[RMAX];
  __shared__ int sh_blk;
  const int tid = threadIdx.x;
  double* scr = g.scratch + (int64_t)blockIdx.x * g.scratch_per_wg;
  double* Qs = scr;                          // BROWS x RMAX, row i at Qs[i*RMAX]
  double* Bs = Qs + BROWS * RMAX;            // B^T: BROWS x RMAX, row j at Bs[j*RMAX]
  double* Gcs = Bs + BROWS * RMAX;           // probes: BROWS x NP
  const double c_alpha = 10.0 * sqrt(2.0 / 3.14159265358979323846);

  for (;;) {
    if (tid == 0) {
      int idx = atomicAdd(g.queue, 1);
      sh_blk = idx < g.nblk ? g.order[idx] : -1;
    }
    __syncthreads();
    const int blk = sh_blk;
    __syncthreads();
    if (blk < 0) break;
    const int m = g.m[blk], n = g.n[blk], lda = g.lda[blk];
    const float* A = g.A[blk];
    if (m < L0 || n < L0 || m > BROWS || n > BROWS || lda < n || A == nullptr) {
      if (tid == 0) { g.rank[blk] = 0; g.status[blk] = -1; }   // invalid block shape
      __syncthreads();
      continue;
    }
    const uint32_t s_om = 16u * (uint32_t)blk + 4u, s_pr = 16u * (uint32_t)blk + 6u;
    const double tau = 16.0 * 1.2e-32;
    const bool row_ok = tid < m, col_ok = tid < n;
    bool nonfinite = false;

    // ---- Y = K [Omega_0 | Gc] (row tid), FP64; the probe part stays as e
    double qv[L0], e[NP];
    {
      double y[L0 + NP];
#pragma unroll
      for (int c = 0; c < L0 + NP; ++c) y[c] = 0.0;
      float* tile = reinterpret_cast<float*>(lds + KC * (L0 + NP));
      for (int j0 = 0; j0 < n; j0 += KC) {
        __syncthreads();
        stage_gauss(lds, L0 + NP, j0, n, L0 + NP, L0, g.seed, s_om, 0, s_pr);
        stage_k(A, lda, m, n, j0, tile);
        __syncthreads();
        for (int t = tid; t < KC * NP; t += BT) {   // keep the probes for B Gc
          int jj = t / NP, c = t - (t / NP) * NP;
          if (j0 + jj < n) Gcs[(j0 + jj) * NP + c] = lds[jj * (L0 + NP) + L0 + c];
        }
        if (row_ok) {
#pragma unroll 2
          for (int jj = 0; jj < KC; ++jj) {
            double a = (double)tile[tid * KLD + jj];
            nonfinite |= !isfinite(a);
#pragma unroll
            for (int c = 0; c < L0 + NP; ++c) y[c] += a * lds[jj * (L0 + NP) + c];
          }
        }
      }
#pragma unroll
      for (int c = 0; c < L0; ++c) qv[c] = row_ok ? y[c] : 0.0;
#pragma unroll
      for (int c = 0; c < NP; ++c) e[c] = row_ok ? y[L0 + c] : 0.0;
    }

    // ---- Q = CholeskyQR2 of Y[:, 0:16]
    for (int pass = 0; pass < 2; ++pass) {
      rows_inner<L0, L0>(qv, L0, qv, L0, m, lds, lds + CH * 2 * L0, L0);
      small_chol_inv<L0>(lds + CH * 2 * L0, lds + CH * 2 * L0 + L0 * L0, Ri, tau);
      double o[L0];
#pragma unroll
      for (int c = 0; c < L0; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < L0; ++a) acc += qv[a] * Ri[a * 16 + c];
        o[c] = acc;
      }
#pragma unroll
      for (int c = 0; c < L0; ++c) qv[c] = o[c];
      __syncthreads();
    }
    if (row_ok)
#pragma unroll
      for (int c = 0; c < L0; ++c) Qs[tid * RMAX + c] = qv[c];

    int rc = 0;   // basis width so far
    double sigma1 = 0.0, bound = 0.0;
    int steps = 0;
    for (;;) {
      const int nw = (rc == 0) ? L0 : BG;   // columns added in this round
      // ---- B_new^T = K^T Q_new (column tid), Q_new rows staged through LDS
      double bt[L0];
#pragma unroll
      for (int c = 0; c < L0; ++c) bt[c] = 0.0;
      for (int i0 = 0; i0 < m; i0 += CH) {
        __syncthreads();
        for (int t = tid; t < CH * L0; t += BT) {
          int ii = t / L0, c = t - (t / L0) * L0;
          lds[ii * L0 + c] = (i0 + ii < m && c < nw) ? Qs[(i0 + ii) * RMAX + rc + c] : 0.0;
        }
        __syncthreads();
        if (col_ok) {
          const int in_ = min(CH, m - i0);
          for (int ii = 0; ii < in_; ++ii) {
            double a = (double)A[(int64_t)(i0 + ii) * lda + tid];
#pragma unroll
            for (int c = 0; c < L0; ++c) bt[c] += a * lds[ii * L0 + c];
          }
        }
      }
      if (col_ok)
#pragma unroll
        for (int c = 0; c < L0; ++c)
          if (c < nw) Bs[tid * RMAX + rc + c] = bt[c];
      // ---- H = B_new Gc (nw x NP); e -= Q_new H
      {
        double gcv[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) gcv[c] = col_ok ? Gcs[tid * NP + c] : 0.0;
        rows_inner<L0, NP>(bt, nw, gcv, NP, n, lds, H, NP);
      }
      if (row_ok) {
        double qn[L0];
#pragma unroll
        for (int c = 0; c < L0; ++c) qn[c] = (c < nw) ? Qs[tid * RMAX + rc + c] : 0.0;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          double acc = 0.0;
#pragma unroll
          for (int c = 0; c < L0; ++c)
            if (c < nw) acc += qn[c] * H[c * NP + b];
          e[b] -= acc;
        }
      }
      rc += nw;
      // ---- bound = 10 sqrt(2/pi) max_b ||e(:, b)||
      double mx = 0.0;
      for (int b = 0; b < NP; ++b) mx = fmax(mx, block_sum(row_ok ? e[b] * e[b] : 0.0, red));
      bound = c_alpha * sqrt(mx);
      if (rc == L0) {
        // sigma_hat_1: largest eigenvalue of B B^T for the first basis
        double* M = lds;
        double* Vm = lds + RMAX * RMAX;
        double br[L0];
#pragma unroll
        for (int c = 0; c < L0; ++c) br[c] = col_ok ? Bs[tid * RMAX + c] : 0.0;
        rows_inner<L0, L0>(br, L0, br, L0, n, lds + 2 * RMAX * RMAX - CH * 2 * L0, H, L0);
        for (int t = tid; t < L0 * L0; t += BT) M[(t / L0) * RMAX + (t % L0)] = H[t];
        __syncthreads();
        small_eig(M, Vm, L0);
        __syncthreads();
        double mxl = 0.0;
        for (int a = 0; a < L0; ++a) mxl = fmax(mxl, M[a * RMAX + a]);
        sigma1 = sqrt(fmax(mxl, 0.0));
        __syncthreads();
      }
      if (bound <= 0.5 * g.eps * sigma1 || rc + BG > min(min(g.rank_cap, RMAX), min(m, n))) break;

      // ---- grow: Y_b = K G_b, projected twice against Q, orthonormalised, appended to Q
      double yb[BG];
#pragma unroll
      for (int c = 0; c < BG; ++c) yb[c] = 0.0;
      float* tile = reinterpret_cast<float*>(lds + KC * BG);
      for (int j0 = 0; j0 < n; j0 += KC) {
        __syncthreads();
        stage_gauss(lds, BG, j0, n, BG, BG, g.seed, s_om, L0 + steps * BG, s_pr);
        stage_k(A, lda, m, n, j0, tile);
        __syncthreads();
        if (row_ok) {
#pragma unroll 2
          for (int jj = 0; jj < KC; ++jj) {
            double a = (double)tile[tid * KLD + jj];
#pragma unroll
            for (int c = 0; c < BG; ++c) yb[c] += a * lds[jj * BG + c];
          }
        }
      }
      for (int pass = 0; pass < 2; ++pass) {
        for (int c0 = 0; c0 < rc; c0 += L0) {   // C = Q^T Y_b in blocks of 16 basis vectors
          double qb[L0];
#pragma unroll
          for (int c = 0; c < L0; ++c) qb[c] = (row_ok && c0 + c < rc) ? Qs[tid * RMAX + c0 + c] : 0.0;
          rows_inner<L0, BG>(qb, L0, yb, BG, m, lds, H, BG);
#pragma unroll
          for (int b = 0; b < BG; ++b) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < L0; ++c) acc += qb[c] * H[c * BG + b];
            yb[b] -= acc;
          }
          __syncthreads();
        }
      }
      for (int pass = 0; pass < 2; ++pass) {
        rows_inner<BG, BG>(yb, BG, yb, BG, m, lds, lds + CH * 2 * BG, BG);
        small_chol_inv<BG>(lds + CH * 2 * BG, lds + CH * 2 * BG + BG * BG, Ri, tau);
        double o[BG];
#pragma unroll
        for (int c = 0; c < BG; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int a = 0; a < BG; ++a) acc += yb[a] * Ri[a * 16 + c];
          o[c] = acc;
        }
#pragma unroll
        for (int c = 0; c < BG; ++c) yb[c] = o[c];
        __syncthreads();
      }
      if (row_ok)
#pragma unroll
        for (int c = 0; c < BG; ++c) Qs[tid * RMAX + rc + c] = yb[c];
      ++steps;
    }

    // ---- SVD of B (rc x n) through the eigen-decomposition of B B^T
    // (with no growth the decomposition made for sigma_hat_1 is still in M, Vm)
    double* M = lds;
    double* Vm = lds + RMAX * RMAX;
    __syncthreads();
    if (rc != L0) {
    for (int t = tid; t < RMAX * RMAX; t += BT) M[t] = 0.0;
    __syncthreads();
    for (int a0 = 0; a0 < rc; a0 += L0)
      for (int b0 = 0; b0 < rc; b0 += L0) {
        double ba[L0], bb[L0];
#pragma unroll
        for (int c = 0; c < L0; ++c) {
          ba[c] = (col_ok && a0 + c < rc) ? Bs[tid * RMAX + a0 + c] : 0.0;
          bb[c] = (col_ok && b0 + c < rc) ? Bs[tid * RMAX + b0 + c] : 0.0;
        }
        rows_inner<L0, L0>(ba, L0, bb, L0, n, Vm, H, L0);   // stage in Vm (free until small_eig)
        for (int t = tid; t < L0 * L0; t += BT) {
          int a = t / L0, b = t % L0;
          if (a0 + a < rc && b0 + b < rc) M[(a0 + a) * RMAX + b0 + b] = H[t];
        }
        __syncthreads();
      }
    small_eig(M, Vm, rc);
    __syncthreads();
    }
    if (tid < rc) {
      double v = M[tid * RMAX + tid];
      int r = 0;
      for (int q = 0; q < rc; ++q) {
        double w = M[q * RMAX + q];
        r += (w > v) || (w == v && q < tid);
      }
      perm[r] = tid;
      sig[r] = sqrt(fmax(v, 0.0));
    }
    __syncthreads();
    const double thr = 0.5 * g.eps * sigma1;
    int keep = 0;
    for (int c = 0; c < rc; ++c) keep += sig[c] > thr;
    keep = min(max(keep, 1), g.rank_cap);
    if (tid < keep) {   // sign rule: entry of largest magnitude of each u_hat column positive
      const int col = perm[tid];
      double best = -1.0, sg = 1.0;
      for (int a = 0; a < rc; ++a) {
        double v = Vm[a * RMAX + col];
        if (fabs(v) > best) { best = fabs(v); sg = v < 0.0 ? -1.0 : 1.0; }
      }
      sgn[tid] = sg;
    }
    __syncthreads();
    // U = Q U_hat(:, :keep), V = B^T U_hat S^-1, S
    float* Uo = g.U + g.offU[blk];
    float* Vo = g.V + g.offV[blk];
    if (row_ok)
      for (int c = 0; c < keep; ++c) {
        const int col = perm[c];
        double acc = 0.0;
        for (int a = 0; a < rc; ++a) acc += Qs[tid * RMAX + a] * Vm[a * RMAX + col];
        Uo[(int64_t)tid * g.rank_cap + c] = (float)(sgn[c] * acc);
      }
    if (col_ok)
      for (int c = 0; c < keep; ++c) {
        const int col = perm[c];
        double acc = 0.0;
        for (int a = 0; a < rc; ++a) acc += Bs[tid * RMAX + a] * Vm[a * RMAX + col];
        Vo[(int64_t)tid * g.rank_cap + c] = (float)(sig[c] > 0.0 ? sgn[c] * acc / sig[c] : 0.0);
      }
    if (tid < keep) g.S[(int64_t)blk * g.rank_cap + tid] = sig[tid];
    const double nf = block_sum(nonfinite ? 1.0 : 0.0, red);
    if (tid == 0) {
      g.rank[blk] = keep;
      g.status[blk] = nf > 0.0 ? -4 : (bound <= 0.5 * g.eps * sigma1 ? 0 : 1);
    }
    __syncthreads();
  }
}

// Largest-first order by a counting sort over 64 size classes of m*n (one workgroup).
__global__ __launch_bounds__(1024) void order_kernel(int nblk, const int* __restrict__ m, const int* __restrict__ n,
                                                     int* __restrict__ order, int* __restrict__ queue) {
  __shared__ int hist[65];
  __shared__ int start[65];
  const int tid = threadIdx.x;
  if (tid < 65) hist[tid] = 0;
  if (tid == 0) *queue = 0;
  __syncthreads();
  for (int b = tid; b < nblk; b += 1024) {
    int64_t sz = (int64_t)m[b] * n[b];
    int cls = 64 - (int)min((int64_t)64, sz >> 12);   // larger blocks first
    atomicAdd(&hist[cls], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int c = 0; c < 65; ++c) { start[c] = acc; acc += hist[c]; }
  }
  __syncthreads();
  for (int b = tid; b < nblk; b += 1024) {
    int64_t sz = (int64_t)m[b] * n[b];
    int cls = 64 - (int)min((int64_t)64, sz >> 12);
    int pos = atomicAdd(&start[cls], 1);
    order[pos] = b;
  }
}

int batched_scratch_doubles_per_wg() { return BROWS * RMAX * 2 + BROWS * NP; }
int batched_max_rank() { return RMAX; }
int batched_max_dim() { return BROWS; }

hipError_t launch_batched(int nblk, const int* m, const int* n, const float* const* A, const int* lda, double eps,
                          int rank_cap, uint64_t seed, float* U, double* S, float* V, const int64_t* offU,
                          const int64_t* offV, int* rank, int* status, int* order, int* queue, double* scratch,
                          int nwg, hipStream_t s) {
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, s, nblk, m, n, order, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchedArgs g{nblk, m, n, A, lda, eps, rank_cap, seed, U, S, V, offU, offV, rank, status, order, queue, scratch,
                (int64_t)batched_scratch_doubles_per_wg()};
  hipLaunchKernelGGL(batched_kernel, dim3((unsigned)nwg), dim3(BT), 0, s, g);
  return hipGetLastError();
}

}  // namespace rsvd
