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
// at eps = 1e-6).
//
// The products with the block -- Y = K [Omega | G_c], B^T = K^T Q, the growth
// sketch K Omega_b -- and the final U = Q U_hat, V = B^T U_hat run on the FP64
// MFMA (mfma_panel below): each wave takes tiles of 16-row groups x 16-column
// groups, streams K straight from memory and the thin panel from the
// workgroup's scratch (L2), with a register ring of prefetched k-slices.  The
// tile shape (row tiles and column tiles per wave task, prefetch depth) is a
// per-size-class parameter picked by the autotuner in batched_api.hip; every
// shape gives bit-identical results.  The small dense steps (16-column Gram
// matrices, Cholesky, the Jacobi eigen-decomposition) stay row-owned: thread t
// owns row t of Y, Q and the probe residual E and column t of B^T, with
// cross-thread sums through 64-row chunks staged in LDS.
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
constexpr int NWAVE = BT / 64;
constexpr int OW = 32;        // columns of the sketch panel [Omega | G_c | 0] and of Y
constexpr int GW = 16;        // columns of the growth panel [Omega_b | 0]
constexpr int NCLASS = 4;     // size classes by max(m, n): (0,128], (128,256], (256,384], (384,512]
constexpr int NVARIANT = 8;   // MFMA tile shapes, see TileShape
constexpr int DEFAULT_VARIANT = 2;

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
  int tile[NCLASS];   // MFMA tile variant per size class
  int class_mask;     // blocks of classes outside the mask are skipped (autotuner timing)
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

// threadIdx.x behind an empty asm: values derived from it cannot be hoisted out
// of the per-block loop.  Without this the compiler precomputes the per-lane
// operand addresses of every inlined product and helper at kernel entry and
// keeps them live (spilled) across the whole persistent loop.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Tile shape of the MFMA products: RT 16-row tiles and NCT 16-column tiles per
// wave task, DEPTH k-slices of 16 in flight.  Variant v: RT = 1 + bit 0,
// NCT = 1 + bit 1, DEPTH = 2 << bit 2.
template <int RT_, int NCT_, int DEPTH_> struct TileShape {
  static constexpr int RT = RT_, NCT = NCT_, DEPTH = DEPTH_;
};

template <typename F> __device__ __forceinline__ void with_tile(int v, F&& f) {
  switch (v) {
    case 0: f(TileShape<1, 1, 2>{}); break;
    case 1: f(TileShape<2, 1, 2>{}); break;
    case 3: f(TileShape<2, 2, 2>{}); break;
    case 4: f(TileShape<1, 1, 4>{}); break;
    case 5: f(TileShape<2, 1, 4>{}); break;
    case 6: f(TileShape<1, 2, 4>{}); break;
    case 7: f(TileShape<2, 2, 4>{}); break;
    default: f(TileShape<1, 2, 2>{}); break;   // variant 2
  }
}

// out = X W on the FP64 MFMA (v_mfma_f64_16x16x4f64).  X is rows x kdim with
// entry (r, k) at X[r*xr + k*xk] (TX = float for the block, double for the
// scratch panels; xr = 1 reads the block transposed); W is kdim x ncols with
// entry (k, c) at W[k*ldw + c].  Entries past rows, kdim or ncols read as zero
// (addresses are clamped, so nothing outside the operands is touched).
// Wave w takes the tasks w, w+8, ... of (RT row tiles) x (NCT column tiles).
// Over each 16-wide k-slice, lane l (g = l/16) feeds data columns k0+4g+s in
// MFMA step s = 0..3, so lane l loads four consecutive k of its row; the
// k-slices are consumed in increasing order by every shape, which makes the
// result of every entry independent of the shape.  epi(r, c, v) receives each
// entry r < rows, c < ncols.
template <typename TX, int RT, int NCT, int DEPTH, typename Epi>
__device__ __forceinline__ void mfma_panel(const TX* __restrict__ X, int64_t xr, int64_t xk, int rows, int kdim,
                                           const double* W, int ldw, int ncols, Epi&& epi) {
  typedef Mma<double> M;
  const int tid = opaque_tid();
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int rgroups = (rows + 16 * RT - 1) / (16 * RT);
  const int cgroups = (ncols + 16 * NCT - 1) / (16 * NCT);
  const int ntask = rgroups * cgroups;
  const int nk = (kdim + 15) >> 4;
  for (int task = wave; task < ntask; task += NWAVE) {
    const int rg = task / cgroups, cg = task - rg * cgroups;
    const TX* xp[RT];
    bool rok[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int r = 16 * (RT * rg + rt) + M::arow(li);
      rok[rt] = r < rows;
      xp[rt] = X + (int64_t)(rok[rt] ? r : 0) * xr;
    }
    int wcol[NCT];
    bool cok[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int c = 16 * (NCT * cg + ct) + li;
      cok[ct] = c < ncols;
      wcol[ct] = cok[ct] ? c : 0;
    }
    typename M::acc acc[RT][NCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = M::zero();
    TX xa[DEPTH][RT][4];
    double wb[DEPTH][NCT][4];
    auto load = [&](int kc, TX(&xs)[RT][4], double(&ws)[NCT][4]) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 16 * kc + 4 * g + s;
        const bool kok = k < kdim;
        const int64_t kk = kok ? k : 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const TX v = xp[rt][kk * xk];
          xs[rt][s] = (kok && rok[rt]) ? v : TX(0);
        }
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const double v = W[kk * ldw + wcol[ct]];
          ws[ct][s] = (kok && cok[ct]) ? v : 0.0;
        }
      }
    };
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) load(d, xa[d], wb[d]);
    for (int kc0 = 0; kc0 < nk; kc0 += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; ++d) {
        if (kc0 + d < nk) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
              for (int ct = 0; ct < NCT; ++ct)
                acc[rt][ct] = M::op((double)xa[d][rt][s], wb[d][ct][s], acc[rt][ct]);
        }
        load(kc0 + d + DEPTH, xa[d], wb[d]);
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int c = 16 * (NCT * cg + ct) + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 16 * (RT * rg + rt) + 4 * g + e;
          if (r < rows && c < ncols) epi(r, c, acc[rt][ct][e]);
        }
      }
  }
}

// Gaussian panel P (ld ldp) for rows [0, n): columns [0, nc0) from stream s0
// starting at column col0, columns [nc0, nc) from stream s1 starting at 0.
// Consecutive threads fill consecutive columns of a row pair.
__device__ void fill_gauss(double* P, int ldp, int n, int nc, int nc0, uint64_t seed, uint32_t s0, int col0,
                           uint32_t s1) {
  const int hp = (n + 1) >> 1;
  for (int t = opaque_tid(); t < hp * nc; t += BT) {
    const int i2 = t / nc, c = t - (t / nc) * nc;
    double z0, z1;
    const bool first = c < nc0;   // one inlined copy of the transform
    bgauss_pair(seed, first ? s0 : s1, (uint32_t)i2, (uint32_t)(first ? col0 + c : c - nc0), z0, z1);
    P[(int64_t)(2 * i2) * ldp + c] = z0;
    if (2 * i2 + 1 < n) P[(int64_t)(2 * i2 + 1) * ldp + c] = z1;
  }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  const int tid = opaque_tid();
  if ((tid & 63) == 0) red[tid >> 6] = v;
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
  const int o = opaque_tid();
  const int a = o / max(nbz, 1), b = o - a * max(nbz, 1);
  for (int r0 = 0; r0 < rows; r0 += CH) {
    __syncthreads();
    if (o >= r0 && o < r0 + CH) {
      const int rr = o - r0;
      const bool ok = o < rows;
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
  const int tid = opaque_tid();
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
  const int tid = opaque_tid();
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
  __shared__ double red[NWAVE * NP];
  __shared__ double sig[RMAX];
  __shared__ double sgn[RMAX];
  __shared__ int perm[RMAX];
  __shared__ int sh_blk;
  double* scr = g.scratch + (int64_t)blockIdx.x * g.scratch_per_wg;
  double* Qs = scr;                          // BROWS x RMAX, row i at Qs[i*RMAX]
  double* Bs = Qs + BROWS * RMAX;            // B^T: BROWS x RMAX, row j at Bs[j*RMAX]
  double* OmG = Bs + BROWS * RMAX;           // [Omega | G_c]: BROWS x OW
  double* Ys = OmG + BROWS * OW;             // sketch outputs: BROWS x OW
  double* Wb = Ys + BROWS * OW;              // growth panel: BROWS x GW
  const double c_alpha = 10.0 * sqrt(2.0 / 3.14159265358979323846);

  for (;;) {
    const int tid = opaque_tid();
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
    const int cls = (max(m, n) - 1) >> 7;
    if (!((g.class_mask >> cls) & 1)) continue;   // uniform: no barrier crossed
    const int tv = g.tile[cls];
    const uint32_t s_om = 16u * (uint32_t)blk + 4u, s_pr = 16u * (uint32_t)blk + 6u;
    const double tau = 16.0 * 1.2e-32;
    const bool row_ok = tid < m, col_ok = tid < n;
    bool nonfinite = false;

    // ---- Y = K [Omega_0 | G_c] on the MFMA; row tid: first 16 columns to qv, probes to e
    fill_gauss(OmG, OW, n, L0 + NP, L0, g.seed, s_om, 0, s_pr);
    __syncthreads();
    with_tile(tv, [&](auto sh) {
      typedef decltype(sh) T;
      mfma_panel<float, T::RT, T::NCT, T::DEPTH>(A, lda, 1, m, n, OmG, OW, L0 + NP,
                                                 [&](int r, int c, double v) { Ys[r * OW + c] = v; });
    });
    __syncthreads();
    double qv[L0], e[NP];
#pragma unroll
    for (int c = 0; c < L0; ++c) qv[c] = row_ok ? Ys[tid * OW + c] : 0.0;
#pragma unroll
    for (int c = 0; c < NP; ++c) e[c] = row_ok ? Ys[tid * OW + L0 + c] : 0.0;
    // every Gaussian entry is nonzero, so a non-finite entry of row tid reaches Y(tid, :)
#pragma unroll
    for (int c = 0; c < L0; ++c) nonfinite |= !isfinite(qv[c]);
#pragma unroll
    for (int c = 0; c < NP; ++c) nonfinite |= !isfinite(e[c]);

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
      // ---- B_new^T = K^T Q_new on the MFMA (rows of B^T are the block's columns)
      __syncthreads();
      with_tile(tv, [&](auto sh) {
        typedef decltype(sh) T;
        mfma_panel<float, T::RT, 1, T::DEPTH>(A, 1, lda, n, m, Qs + rc, RMAX, nw, [&](int j, int c, double v) {
          Bs[j * RMAX + rc + c] = v;
        });
      });
      __syncthreads();
      double bt[L0];
#pragma unroll
      for (int c = 0; c < L0; ++c) bt[c] = (col_ok && c < nw) ? Bs[tid * RMAX + rc + c] : 0.0;
      // ---- H = B_new Gc (nw x NP); e -= Q_new H
      {
        double gcv[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) gcv[c] = col_ok ? OmG[tid * OW + L0 + c] : 0.0;
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
      // ---- bound = 10 sqrt(2/pi) max_b ||e(:, b)||: the NP column sums in one reduction
      {
        double ss[NP];
#pragma unroll
        for (int b = 0; b < NP; ++b) ss[b] = wave_sum(row_ok ? e[b] * e[b] : 0.0);
        if ((tid & 63) == 0)
#pragma unroll
          for (int b = 0; b < NP; ++b) red[(tid >> 6) * NP + b] = ss[b];
        __syncthreads();
        double mx = 0.0;
        for (int b = 0; b < NP; ++b) {
          double t = 0.0;
#pragma unroll
          for (int w = 0; w < NWAVE; ++w) t += red[w * NP + b];
          mx = fmax(mx, t);
        }
        bound = c_alpha * sqrt(mx);
      }
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
      }
      __syncthreads();
      if (bound <= 0.5 * g.eps * sigma1 || rc + BG > min(min(g.rank_cap, RMAX), min(m, n))) break;

      // ---- grow: Y_b = K Omega_b on the MFMA, projected twice against Q, orthonormalised, appended
      fill_gauss(Wb, GW, n, BG, BG, g.seed, s_om, L0 + steps * BG, s_pr);
      __syncthreads();
      with_tile(tv, [&](auto sh) {
        typedef decltype(sh) T;
        mfma_panel<float, T::RT, 1, T::DEPTH>(A, lda, 1, m, n, Wb, GW, BG,
                                              [&](int r, int c, double v) { Ys[r * OW + c] = v; });
      });
      __syncthreads();
      double yb[BG];
#pragma unroll
      for (int c = 0; c < BG; ++c) yb[c] = row_ok ? Ys[tid * OW + c] : 0.0;
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
    // W = U_hat(:, perm[:keep]) with the signs applied, over M (free now)
    double* Wu = M;
    for (int t = tid; t < RMAX * RMAX; t += BT) {
      const int a = t / RMAX, c = t - (t / RMAX) * RMAX;
      Wu[t] = (a < rc && c < keep) ? sgn[c] * Vm[a * RMAX + perm[c]] : 0.0;
    }
    __syncthreads();
    // U = Q W, V = B^T W S^-1, S
    float* Uo = g.U + g.offU[blk];
    float* Vo = g.V + g.offV[blk];
    const int rcap = g.rank_cap;
    mfma_panel<double, 1, 1, 2>(Qs, RMAX, 1, m, rc, Wu, RMAX, keep, [&](int r, int c, double v) {
      Uo[(int64_t)r * rcap + c] = (float)v;
    });
    mfma_panel<double, 1, 1, 2>(Bs, RMAX, 1, n, rc, Wu, RMAX, keep, [&](int j, int c, double v) {
      Vo[(int64_t)j * rcap + c] = (float)(sig[c] > 0.0 ? v / sig[c] : 0.0);
    });
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
  const int tid = opaque_tid();
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

int batched_scratch_doubles_per_wg() { return BROWS * (2 * RMAX + 2 * OW + GW); }
int batched_num_classes() { return NCLASS; }
int batched_num_variants() { return NVARIANT; }
int batched_default_variant() { return DEFAULT_VARIANT; }
int batched_max_rank() { return RMAX; }
int batched_max_dim() { return BROWS; }

int batched_resident_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_kernel, BT, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_batched(int nblk, const int* m, const int* n, const float* const* A, const int* lda, double eps,
                          int rank_cap, uint64_t seed, float* U, double* S, float* V, const int64_t* offU,
                          const int64_t* offV, int* rank, int* status, int* order, int* queue, double* scratch,
                          int nwg, const int* tiles, int class_mask, hipStream_t s) {
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, s, nblk, m, n, order, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchedArgs g{nblk, m, n, A, lda, eps, rank_cap, seed, U, S, V, offU, offV, rank, status, order, queue, scratch,
                (int64_t)batched_scratch_doubles_per_wg(), {}, class_mask};
  for (int c = 0; c < NCLASS; ++c) {
    const int v = tiles ? tiles[c] : DEFAULT_VARIANT;
    if (v < 0 || v >= NVARIANT) return hipErrorInvalidValue;
    g.tile[c] = v;
  }
  hipLaunchKernelGGL(batched_kernel, dim3((unsigned)nwg), dim3(BT), 0, s, g);
  return hipGetLastError();
}

}  // namespace rsvd
