// Skinny products with the large matrix A on MFMA (gfx950).
//
// Every heavy step of the method is a product of the m x n matrix A (or a
// tall l-column panel) with a thin panel of at most a few hundred columns:
//   sketch   Y = A Omega,  power step  Y = A W          (nn_kernel, K = n)
//   power    Z = A^T Q,    projection  B^T = A^T Q      (tn_kernel, K = m)
//   Gram     G = Y^T Y   (nn_kernel with A := Y^T, split over the rows)
//   triangular apply Q = Y R^-1 and the lifts U = Q U_hat, V = B^T (U_hat D^-1)
//                       (tn_kernel with A := Y^T)
// Thin panels live in HBM in "panel" layout: column c is contiguous
// (element (r, c) at p[c * ld + r], ld a multiple of 64), so a panel is the
// row-major transpose of the tall matrix.
//
// Design (both kernels):
//   * 256 threads = 4 wave64s; the thin panel's K-chunk (64 rows) is staged in
//     LDS in MFMA-fragment order, so each lane reads its B operand with one
//     16-byte ds_read and every wave of the block shares it;
//   * A is read straight from HBM into registers, 16 bytes per lane per load:
//     the contraction index is permuted within each 16-wide K group so a lane
//     holds four consecutive K entries of one row (nn) or four consecutive
//     output rows of one K entry (tn), exactly what the 16x16x4 MFMA consumes
//     over four instructions;
//   * each block covers a full panel-column group (up to 128 columns), so A is
//     read once per group; the K range is split over grid.y and partial
//     results are summed afterwards in a fixed order (deterministic, no
//     atomics).
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace rsvd {

constexpr int KC = 64;   // K rows staged per iteration

// Stage panel rows [k0, k0+64) of columns [cg0, cg0+NB*16) of a panel P
// (column c contiguous, stride ldp) into LDS fragment order:
//   ps[(cb*4 + kq)*64 + (c%16) + 16*g].x[t] = P(c, k0 + 16*kq + 4*g + t).
template <int NB, typename TP, typename TC>
__device__ __forceinline__ void stage_panel(V4<TC>* ps, const TP* __restrict__ P, int64_t ldp, int cg0, int ncols,
                                            int64_t k0, int64_t kend) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    int it = threadIdx.x + 256 * u;
    int cl = it >> 4, jq = it & 15;
    int c = cg0 + cl;
    V4<TP> v = (c < ncols) ? load4_guarded<true>(P, ldp, (int64_t)c, k0 + 4 * jq, (int64_t)ncols, kend)
                           : v4_zero<TP>();
    int cb = cl >> 4, cli = cl & 15, kq = jq >> 2, g = jq & 3;
    ps[(cb * 4 + kq) * 64 + cli + 16 * g] = v4_cast<TC>(v);
  }
}

// The two halves of stage_panel: this thread's NB values of the chunk into registers, and from there into LDS.
template <int NB, typename TP>
__device__ __forceinline__ void panel_load(V4<TP> (&v)[NB], const TP* __restrict__ P, int64_t ldp, int cg0, int ncols,
                                           int64_t k0, int64_t kend) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    int it = threadIdx.x + 256 * u;
    int cl = it >> 4, jq = it & 15;
    int c = cg0 + cl;
    v[u] = (c < ncols) ? load4_guarded<true>(P, ldp, (int64_t)c, k0 + 4 * jq, (int64_t)ncols, kend) : v4_zero<TP>();
  }
}
template <int NB, typename TP, typename TC>
__device__ __forceinline__ void panel_store(V4<TC>* ps, const V4<TP> (&v)[NB]) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    int it = threadIdx.x + 256 * u;
    int cl = it >> 4, jq = it & 15;
    int cb = cl >> 4, cli = cl & 15, kq = jq >> 2, g = jq & 3;
    ps[(cb * 4 + kq) * 64 + cli + 16 * g] = v4_cast<TC>(v[u]);
  }
}

// out[split][c][r] = sum_{j in split} A[r][j] * X(j, c)      (X in panel layout: X[c*ldx + j]), FP32 operands:
// software-pipelined, the next chunk's A values and panel values are loaded into registers while the current
// chunk is multiplied, the panel going to the spare of two LDS buffers (one barrier per chunk).
template <typename TX, typename TO, int NB, bool VEC>
__global__ __launch_bounds__(256) void nn_pipe_kernel(const float* __restrict__ A, int64_t lda, int64_t rows,
                                                      int64_t K, const TX* __restrict__ X, int64_t ldx, int ncols,
                                                      TO* __restrict__ out, int64_t ldo, int64_t part_stride,
                                                      int64_t kchunk, int cg_off) {
  __shared__ V4<float> xs[2][NB * 4 * 64];
  typedef Mma<float> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * 128 + wave * 32;
  const int split = blockIdx.y;
  const int cg0 = cg_off + blockIdx.z * NB * 16;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);

  typename M::acc acc[2][NB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = M::zero();

  V4<float> a[2][4];
  V4<TX> xr[NB];
  auto load_a = [&](V4<float> (&dst)[2][4], int64_t k0) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int kq = 0; kq < 4; ++kq)
        dst[rb][kq] = load4_guarded<VEC>(A, lda, rbase + 16 * rb + M::arow(li), k0 + 16 * kq + 4 * g, rows, kend);
  };
  if (kbeg < kend) {
    load_a(a, kbeg);
    panel_load<NB>(xr, X, ldx, cg0, ncols, kbeg, kend);
    panel_store<NB, TX, float>(xs[0], xr);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    const bool more = k0 + KC < kend;   // uniform
    V4<float> an[2][4];
    if (more) {
      load_a(an, k0 + KC);
      panel_load<NB>(xr, X, ldx, cg0, ncols, k0 + KC, kend);
    }
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      V4<float> b[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) b[cb] = xs[cur][(cb * 4 + kq) * 64 + lane];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const float av = a[rb][kq].x[t];
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = M::op(av, b[cb].x[t], acc[rb][cb]);
        }
    }
    if (more) panel_store<NB, TX, float>(xs[cur ^ 1], xr);
    __syncthreads();
    if (more) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) a[rb][kq] = an[rb][kq];
    }
    cur ^= 1;
  }

  TO* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      int c = cg0 + cb * 16 + li;
      if (c >= ncols) continue;
      int64_t r = rbase + rb * 16 + 4 * g;
      TO* p = o + (int64_t)c * ldo + r;
      if (r + 4 <= rows) {
        V4<TO> v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v.x[e] = static_cast<TO>(acc[rb][cb][e]);
        v4_store(p, v);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (r + e < rows) p[e] = static_cast<TO>(acc[rb][cb][e]);
      }
    }
}

// out[split][c][r] = sum_{j in split} A[r][j] * X(j, c)      (X in panel layout: X[c*ldx + j])
template <typename TA, typename TX, typename TC, typename TO, int NB, bool VEC>
__global__ __launch_bounds__(256) void nn_kernel(const TA* __restrict__ A, int64_t lda, int64_t rows, int64_t K,
                                                 const TX* __restrict__ X, int64_t ldx, int ncols,
                                                 TO* __restrict__ out, int64_t ldo, int64_t part_stride,
                                                 int64_t kchunk, int cg_off) {
  __shared__ V4<TC> xs[NB * 4 * 64];
  typedef Mma<TC> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * 128 + wave * 32;
  const int split = blockIdx.y;
  const int cg0 = cg_off + blockIdx.z * NB * 16;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);

  typename M::acc acc[2][NB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = M::zero();

  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    stage_panel<NB>(xs, X, ldx, cg0, ncols, k0, kend);
    V4<TA> a[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int kq = 0; kq < 4; ++kq)
        a[rb][kq] = load4_guarded<VEC>(A, lda, rbase + 16 * rb + M::arow(li), k0 + 16 * kq + 4 * g, rows, kend);
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      V4<TC> b[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) b[cb] = xs[(cb * 4 + kq) * 64 + lane];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          TC av = static_cast<TC>(a[rb][kq].x[t]);
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = M::op(av, b[cb].x[t], acc[rb][cb]);
        }
    }
    __syncthreads();
  }

  TO* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      int c = cg0 + cb * 16 + li;
      if (c >= ncols) continue;
      int64_t r = rbase + rb * 16 + 4 * g;
      TO* p = o + (int64_t)c * ldo + r;
      if (r + 4 <= rows) {
        V4<TO> v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v.x[e] = static_cast<TO>(acc[rb][cb][e]);
        v4_store(p, v);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (r + e < rows) p[e] = static_cast<TO>(acc[rb][cb][e]);
      }
    }
}

// tn_kernel for FP32 operands, software-pipelined like nn_pipe_kernel: the next chunk's A values (16 loads of
// four per lane) and panel values are loaded into registers while the current chunk is multiplied.
template <typename TP, typename TO, int NB, bool VEC, bool OUT_RM>
__global__ __launch_bounds__(256) void tn_pipe_kernel(const float* __restrict__ A, int64_t lda, int64_t K, int64_t N,
                                                      const TP* __restrict__ P, int64_t ldp, int ncols,
                                                      TO* __restrict__ out, int64_t ldo, int64_t part_stride,
                                                      int64_t kchunk, bool upper, TO* __restrict__ out_skip,
                                                      const int* __restrict__ skip, int cg_off) {
  if (skip && *skip) {   // a skipped second CholeskyQR pass (uniform): write elsewhere, or nothing
    if (!out_skip) return;
    out = out_skip;
  }
  __shared__ V4<float> ps[2][NB * 4 * 64];
  typedef Mma<float> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t jw = (int64_t)blockIdx.x * 256 + wave * 64;   // this wave's 64 output rows
  const int split = blockIdx.y;
  const int cg0 = cg_off + blockIdx.z * NB * 16;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = upper ? min(min(K, kbeg + kchunk), (int64_t)cg0 + NB * 16) : min(K, kbeg + kchunk);

  // acc[bb][cb]: MFMA tile row m <-> output row jw + 4*arow(m) + bb
  typename M::acc acc[4][NB];
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[bb][cb] = M::zero();

  V4<float> a[4][4];
  V4<TP> xr[NB];
  auto load_a = [&](V4<float> (&dst)[4][4], int64_t k0) {
#pragma unroll
    for (int kq = 0; kq < 4; ++kq)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        dst[kq][t] = load4_guarded<VEC>(A, lda, k0 + 16 * kq + 4 * g + t, jw + 4 * M::arow(li), kend, N);
  };
  if (kbeg < kend) {
    load_a(a, kbeg);
    panel_load<NB>(xr, P, ldp, cg0, ncols, kbeg, kend);
    panel_store<NB, TP, float>(ps[0], xr);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    const bool more = k0 + KC < kend;   // uniform
    V4<float> an[4][4];
    if (more) {
      load_a(an, k0 + KC);
      panel_load<NB>(xr, P, ldp, cg0, ncols, k0 + KC, kend);
    }
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      V4<float> b[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) b[cb] = ps[cur][(cb * 4 + kq) * 64 + lane];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          const float av = a[kq][t].x[bb];
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) acc[bb][cb] = M::op(av, b[cb].x[t], acc[bb][cb]);
        }
    }
    if (more) panel_store<NB, TP, float>(ps[cur ^ 1], xr);
    __syncthreads();
    if (more) {
#pragma unroll
      for (int kq = 0; kq < 4; ++kq)
#pragma unroll
        for (int t = 0; t < 4; ++t) a[kq][t] = an[kq][t];
    }
    cur ^= 1;
  }

  TO* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    int c = cg0 + cb * 16 + li;
    if (c >= ncols) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int64_t j = jw + 16 * g + 4 * r;   // rows j .. j+3 <-> bb = 0..3
      if (OUT_RM) {
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          if (j + bb < N) o[(j + bb) * ldo + c] = static_cast<TO>(acc[bb][cb][r]);
      } else {
        TO* p = o + (int64_t)c * ldo + j;
        if (j + 4 <= N) {
          V4<TO> v;
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) v.x[bb] = static_cast<TO>(acc[bb][cb][r]);
          v4_store(p, v);
        } else {
#pragma unroll
          for (int bb = 0; bb < 4; ++bb)
            if (j + bb < N) p[bb] = static_cast<TO>(acc[bb][cb][r]);
        }
      }
    }
  }
}

// out[split][c][j] = sum_{i in split} A[i][j] * P(i, c)      (P in panel layout: P[c*ldp + i])
// OUT_RM: write out[j*ldo + c] instead (row-major result, no split).
// upper: P is upper triangular (P(i, c) = 0 for i > c), so a column group stops at its last column.
template <typename TA, typename TP, typename TC, typename TO, int NB, bool VEC, bool OUT_RM>
__global__ __launch_bounds__(256) void tn_kernel(const TA* __restrict__ A, int64_t lda, int64_t K, int64_t N,
                                                 const TP* __restrict__ P, int64_t ldp, int ncols,
                                                 TO* __restrict__ out, int64_t ldo, int64_t part_stride,
                                                 int64_t kchunk, bool upper, TO* __restrict__ out_skip,
                                                 const int* __restrict__ skip, int cg_off) {
  if (skip && *skip) {   // a skipped second CholeskyQR pass (uniform): write elsewhere, or nothing
    if (!out_skip) return;
    out = out_skip;
  }
  __shared__ V4<TC> ps[NB * 4 * 64];
  typedef Mma<TC> M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t jw = (int64_t)blockIdx.x * 256 + wave * 64;   // this wave's 64 output rows
  const int split = blockIdx.y;
  const int cg0 = cg_off + blockIdx.z * NB * 16;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = upper ? min(min(K, kbeg + kchunk), (int64_t)cg0 + NB * 16) : min(K, kbeg + kchunk);

  // acc[bb][cb]: MFMA tile row m <-> output row jw + 4*arow(m) + bb
  typename M::acc acc[4][NB];
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[bb][cb] = M::zero();

  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    stage_panel<NB>(ps, P, ldp, cg0, ncols, k0, kend);
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      V4<TA> a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        a[t] = load4_guarded<VEC>(A, lda, k0 + 16 * kq + 4 * g + t, jw + 4 * M::arow(li), kend, N);
      V4<TC> b[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) b[cb] = ps[(cb * 4 + kq) * 64 + lane];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          TC av = static_cast<TC>(a[t].x[bb]);
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) acc[bb][cb] = M::op(av, b[cb].x[t], acc[bb][cb]);
        }
    }
    __syncthreads();
  }

  TO* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    int c = cg0 + cb * 16 + li;
    if (c >= ncols) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int64_t j = jw + 16 * g + 4 * r;   // rows j .. j+3 <-> bb = 0..3
      if (OUT_RM) {
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          if (j + bb < N) o[(j + bb) * ldo + c] = static_cast<TO>(acc[bb][cb][r]);
      } else {
        TO* p = o + (int64_t)c * ldo + j;
        if (j + 4 <= N) {
          V4<TO> v;
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) v.x[bb] = static_cast<TO>(acc[bb][cb][r]);
          v4_store(p, v);
        } else {
#pragma unroll
          for (int bb = 0; bb < 4; ++bb)
            if (j + bb < N) p[bb] = static_cast<TO>(acc[bb][cb][r]);
        }
      }
    }
  }
}

// out[c*ldo + r] = sum_{s < S} part[s*ps + c*ldp + r]  (fixed order), r < rows, c < ncols.
// grid.y = group: partials [group*S, min((group+1)*S, Stot)) go to out + group*ostride.
template <typename TP, typename TO>
__global__ __launch_bounds__(256) void reduce_kernel(const TP* __restrict__ part, int S, int Stot, int64_t pstride,
                                                     int64_t ldp, int64_t rows, int ncols, TO* __restrict__ out,
                                                     int64_t ldo, int64_t ostride, const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t nq = (rows + 3) / 4;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nq * ncols) return;
  const int s0 = blockIdx.y * S;
  const int cnt = min(S, Stot - s0);
  int64_t c = t / nq, r = 4 * (t % nq);
  const TP* p = part + (int64_t)s0 * pstride + c * ldp + r;
  TO* o = out + blockIdx.y * ostride + c * ldo + r;
  if (r + 4 <= rows) {
    // eight partials loaded ahead of their (in-order) additions, so the loads overlap; past the last
    // partial a batch re-reads it (clamped index) and adds zero
    V4<TP> s = v4_load(p);
    for (int k = 1; k < cnt; k += 8) {
      V4<TP> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = v4_load(p + (int64_t)min(k + u, cnt - 1) * pstride);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) s.x[e] += (k + u < cnt) ? v[u].x[e] : TP(0);
    }
    v4_store(o, v4_cast<TO>(s));
  } else {
    for (int e = 0; r + e < rows; ++e) {
      TP s = p[e];
      for (int k = 1; k < cnt; ++k) s += p[k * pstride + e];
      o[e] = static_cast<TO>(s);
    }
  }
}

// out[c*ldo + r] = sum_{s < S} part[s*ps + c*ldp + r] in one launch, for many partials of a small
// result: a workgroup takes 64 consecutive entries and 16 partial groups; thread (entry e, group q) adds
// partials q, q + 16, q + 32, ... of its entry in that order (eight loads ahead of the additions), then the
// 16 group sums are added in order q = 0 .. 15 (a fixed order: deterministic).
template <typename TP>
__global__ __launch_bounds__(1024) void reduce_tree_kernel(const TP* __restrict__ part, int S, int64_t pstride,
                                                           int64_t ldp, int64_t rows, int ncols,
                                                           TP* __restrict__ out, int64_t ldo,
                                                           const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ TP red[16][64];
  const int e = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t n = rows * ncols;
  const int64_t idx = (int64_t)blockIdx.x * 64 + e;
  const int64_t ii = idx < n ? idx : n - 1;   // past the end: a valid entry, never stored
  const int64_t c = ii / rows, r = ii - (ii / rows) * rows;
  const TP* p = part + c * ldp + r;
  TP acc = TP(0);
  for (int k = q; k < S; k += 16 * 8) {
    TP v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)min(k + 16 * u, S - 1) * pstride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (k + 16 * u < S) ? v[u] : TP(0);
  }
  red[q][e] = acc;
  __syncthreads();
  if (q == 0 && idx < n) {
    TP t = red[0][e];
#pragma unroll
    for (int j = 1; j < 16; ++j) t += red[j][e];
    out[c * ldo + r] = t;
  }
}

// ------------------------------------------------------------------ launchers

static inline int nb_for(int ncols) { int nb = (ncols + 15) / 16; return nb > 8 ? 8 : (nb < 1 ? 1 : nb); }

#define RSVD_NB_SWITCH(NBV, ...)                          \
  switch (NBV) {                                          \
    case 1: { constexpr int NB = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NB = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int NB = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int NB = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int NB = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int NB = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int NB = 7; __VA_ARGS__; } break; \
    default: { constexpr int NB = 8; __VA_ARGS__; } break; \
  }

template <typename TA, typename TX, typename TC, typename TO>
hipError_t launch_nn(const TA* A, int64_t lda, int64_t rows, int64_t K, const TX* X, int64_t ldx, int ncols,
                     TO* out, int64_t ldo, int64_t part_stride, int splits, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + KC - 1) / KC * KC;
  if (kchunk < KC) kchunk = KC;
  int used = (int)((K + kchunk - 1) / kchunk);
  if (used < 1) used = 1;
  const int nb = nb_for(ncols);
  const int groups = (ncols + nb * 16 - 1) / (nb * 16);
  dim3 grid((unsigned)((rows + 127) / 128), (unsigned)used, (unsigned)groups);
  bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  // a last column group with fewer live blocks than the others goes to a launch of its own with only those
  // blocks (at 520 columns: four groups of 8 blocks, then one of 1, instead of five of 8)
  const int nb_last = (ncols - 16 * nb * (groups - 1) + 15) / 16;
  const bool split_last = groups > 1 && nb_last < nb;
  for (int part = 0; part < (split_last ? 2 : 1); ++part) {
    const int nbv = part == 1 ? nb_last : nb;
    const int cg_off = part == 1 ? 16 * nb * (groups - 1) : 0;
    grid.z = (unsigned)(part == 1 ? 1 : split_last ? groups - 1 : groups);
    if constexpr (std::is_same<TA, float>::value && std::is_same<TC, float>::value) {
      RSVD_NB_SWITCH(nbv, {
        if (vec)
          hipLaunchKernelGGL((nn_pipe_kernel<TX, TO, NB, true>), grid, dim3(256), 0, s, A, lda, rows, K, X, ldx,
                             ncols, out, ldo, part_stride, kchunk, cg_off);
        else
          hipLaunchKernelGGL((nn_pipe_kernel<TX, TO, NB, false>), grid, dim3(256), 0, s, A, lda, rows, K, X, ldx,
                             ncols, out, ldo, part_stride, kchunk, cg_off);
      });
    } else {
      RSVD_NB_SWITCH(nbv, {
        if (vec)
          hipLaunchKernelGGL((nn_kernel<TA, TX, TC, TO, NB, true>), grid, dim3(256), 0, s, A, lda, rows, K, X, ldx,
                             ncols, out, ldo, part_stride, kchunk, cg_off);
        else
          hipLaunchKernelGGL((nn_kernel<TA, TX, TC, TO, NB, false>), grid, dim3(256), 0, s, A, lda, rows, K, X, ldx,
                             ncols, out, ldo, part_stride, kchunk, cg_off);
      });
    }
  }
  return hipGetLastError();
}

int nn_splits_used(int64_t K, int splits) {
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + KC - 1) / KC * KC;
  if (kchunk < KC) kchunk = KC;
  int used = (int)((K + kchunk - 1) / kchunk);
  return used < 1 ? 1 : used;
}

// Short contractions (K <= 128, ncols <= 128; A FP32, P and out FP32 or FP64): out[c*ldo + j] (or
// out[j*ldo + c], row-major) =
// sum_{i < K} A[i*lda + j] * P(i, c), as tn_kernel with one range, for the apply X <- X R^-1 of
// CholeskyQR and the lifts U = Q U_hat, V = B^T V_hat (K = l).  The whole of P
// goes to LDS once per workgroup as 128 rows (rows K .. 127 zero, so every task runs the same 32
// MFMA steps with no branches; pitch 144 elements so that the four k-rows a B fragment reads fall on
// different banks); a wave takes 16-row tasks (all columns at once) and loads the task's A slice
// in full before its MFMAs, prefetching the next task's slice meanwhile.  One workgroup per
// compute unit: more workgroups only repeat the staging of P (measured: 512 or 1024 workgroups
// of 256 threads, or 256 of 512 threads, are all slower at l = 110).
// Every A load is unconditional: rows past N are clamped (their outputs are not stored) and k past
// K is clamped (it meets a zero row of P).
constexpr int kApplyPitch = 144;
constexpr int kApplyKMax = 128;
constexpr int kApplyThreads = 256;   // 4 waves; one workgroup per compute unit stages P once

// TRI: P is upper triangular (P(i, c) = 0 for i > c, as R^-1 is), so column tile ct takes only the
// k-steps s < 4 (ct + 1); the loops are unrolled, so the skip costs no branch.
// TP = double: P, the accumulation and the output in FP64 (A converted exactly); the FP64 MFMA puts
// A lane arow(m) at accumulator row m, so a lane loads row arow(li) and the stores are as for FP32.
template <typename TP, int NCT, bool TRI>
__global__ __launch_bounds__(kApplyThreads) void apply_small_kernel(const float* __restrict__ A, int64_t lda, int K, int64_t N,
                                                          const TP* __restrict__ P, int64_t ldp, int ncols,
                                                          TP* __restrict__ out, int64_t ldo, bool vec_out,
                                                          bool rowmajor, TP* __restrict__ out_skip,
                                                          const int* __restrict__ skip) {
  if (skip && *skip) {   // a skipped second CholeskyQR pass (uniform): write elsewhere, or nothing
    if (!out_skip) return;
    out = out_skip;
  }
  constexpr int KS = kApplyKMax / 4;   // MFMA k-steps of a task at most
  __shared__ TP ps[kApplyKMax * kApplyPitch];
  typedef Mma<TP> M;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, li = lane & 15;
  {
    // all loads first (unconditional, clamped indices), then the LDS stores: a guarded load per
    // iteration would wait for each load in turn.  Rows K .. 127 are zeroed by a 0/1 factor
    // (P is finite), columns past ncols are never read by a stored output.
    constexpr int PER = kApplyKMax * kApplyKMax / kApplyThreads;
    constexpr int total = kApplyKMax * NCT * 16;   // all 128 rows: those past K are zero
    TP v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = min(tid + kApplyThreads * u, total - 1);   // consecutive threads: consecutive k of a column
      const int c = t / kApplyKMax, i = t - c * kApplyKMax;
      v[u] = P[(uint32_t)(min(c, ncols - 1) * (uint32_t)ldp + min(i, K - 1))];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = tid + kApplyThreads * u;
      const int c = t / kApplyKMax, i = t - c * kApplyKMax;
      if (t < total) ps[i * kApplyPitch + c] = v[u] * (i < K ? TP(1) : TP(0));
    }
  }
  __syncthreads();
  const int64_t ntask = (N + 15) / 16;
  const int64_t stride = (int64_t)gridDim.x * (kApplyThreads / 64);
  int64_t task = (int64_t)blockIdx.x * (kApplyThreads / 64) + wave;
  TP a[KS];
  // 32-bit offsets from the scalar base (K * lda < 2^32 is checked at launch): one VGPR per address
  const int lrow = sizeof(TP) == 8 ? Mma<double>::arow(li) : li;
  auto load = [&](int64_t tk, TP(&av)[KS]) {
    const uint32_t j = (uint32_t)min(tk * 16 + lrow, N - 1);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const uint32_t i = (uint32_t)min(4 * s + g, K - 1);
      av[s] = static_cast<TP>(A[i * (uint32_t)lda + j]);
    }
  };
  auto compute = [&](int64_t tk, const TP(&av)[KS]) {
    typename M::acc acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = M::zero();
#pragma unroll
    for (int s = 0; s < KS; ++s) {   // every step: rows past K of P are zero in LDS (no branches)
      const TP* pr = ps + (4 * s + g) * kApplyPitch + li;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        if (!TRI || s < 4 * (ct + 1)) acc[ct] = M::op(av[s], pr[16 * ct], acc[ct]);
    }
    const int64_t j = tk * 16 + 4 * g;   // rows j .. j+3 <-> accumulator elements 0..3
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int c = 16 * ct + li;
      if (c >= ncols) continue;
      if (rowmajor) {   // out[j * ldo + c]: 16 consecutive columns per row and instruction
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (j + r < N) out[(j + r) * ldo + c] = acc[ct][r];
        continue;
      }
      TP* p = out + (int64_t)c * ldo + j;
      if (vec_out && j + 4 <= N) {
        V4<TP> v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v.x[r] = acc[ct][r];
        v4_store(p, v);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (j + r < N) p[r] = acc[ct][r];
      }
    }
  };
  // two tasks per iteration with fixed buffers: the next task's slice loads during the products
  TP a2[KS];
  if (task < ntask) load(task, a);
  for (; task < ntask; task += 2 * stride) {
    const int64_t t1 = task + stride;
    if (t1 < ntask) load(t1, a2);
    compute(task, a);
    if (t1 >= ntask) break;
    if (t1 + stride < ntask) load(t1 + stride, a);
    compute(t1, a2);
  }
}

template <typename TP>
hipError_t launch_apply_small(const float* A, int64_t lda, int K, int64_t N, const TP* P, int64_t ldp, int ncols,
                              TP* out, int64_t ldo, bool tri, bool rowmajor, hipStream_t s, TP* out_skip = nullptr,
                              const int* skip = nullptr) {
  const int nct = (ncols + 15) / 16;
  const int64_t ntask = (N + 15) / 16;
  const int wpg = kApplyThreads / 64;
  const unsigned grid = (unsigned)std::min<int64_t>((ntask + wpg - 1) / wpg, 256);   // each workgroup stages P once
  const bool vec = (ldo % 4 == 0) && ((reinterpret_cast<uintptr_t>(out) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(out_skip) & 15) == 0);
  switch (nct) {
#define RSVD_APPLY_CASE(N_)                                                                                       \
  case N_:                                                                                                        \
    if (tri)                                                                                                      \
      hipLaunchKernelGGL((apply_small_kernel<TP, N_, true>), dim3(grid), dim3(kApplyThreads), 0, s, A, lda, K, N, P, \
                         ldp, ncols, out, ldo, vec, rowmajor, out_skip, skip);                                    \
    else                                                                                                          \
      hipLaunchKernelGGL((apply_small_kernel<TP, N_, false>), dim3(grid), dim3(kApplyThreads), 0, s, A, lda, K, N, \
                         P, ldp, ncols, out, ldo, vec, rowmajor, out_skip, skip);                                 \
    break;
    RSVD_APPLY_CASE(1) RSVD_APPLY_CASE(2) RSVD_APPLY_CASE(3) RSVD_APPLY_CASE(4)
    RSVD_APPLY_CASE(5) RSVD_APPLY_CASE(6) RSVD_APPLY_CASE(7) RSVD_APPLY_CASE(8)
#undef RSVD_APPLY_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TA, typename TP, typename TC, typename TO>
static hipError_t launch_tn_k(const TA* A, int64_t lda, int64_t K, int64_t N, const TP* P, int64_t ldp, int ncols,
                              TO* out, int64_t ldo, int64_t part_stride, int splits, bool out_rowmajor, bool upper,
                              hipStream_t s, const int* skip = nullptr, TO* out_skip = nullptr) {
  if (N <= 0 || ncols <= 0) return hipSuccess;
  if (splits < 1 || out_rowmajor) splits = 1;
  if constexpr (std::is_same<TA, float>::value && std::is_same<TP, float>::value && std::is_same<TO, float>::value &&
                std::is_same<TC, float>::value) {
    if (splits == 1 && K <= kApplyKMax && ncols <= kApplyKMax && K * lda < (int64_t(1) << 32) &&
        (int64_t)ncols * ldp < (int64_t(1) << 32))
      return launch_apply_small(A, lda, (int)K, N, P, ldp, ncols, out, ldo, upper, out_rowmajor, s, out_skip, skip);
  }
  int64_t kchunk = ((K + splits - 1) / splits + KC - 1) / KC * KC;
  if (kchunk < KC) kchunk = KC;
  int used = (int)((K + kchunk - 1) / kchunk);
  if (used < 1) used = 1;
  const int nb = nb_for(ncols);
  const int groups = (ncols + nb * 16 - 1) / (nb * 16);
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)used, (unsigned)groups);
  bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  // a last column group with fewer live blocks than the others: a launch of its own with only those blocks
  const int nb_last = (ncols - 16 * nb * (groups - 1) + 15) / 16;
  const bool split_last = groups > 1 && nb_last < nb;
  for (int part = 0; part < (split_last ? 2 : 1); ++part) {
    const int nbv = part == 1 ? nb_last : nb;
    const int cg_off = part == 1 ? 16 * nb * (groups - 1) : 0;
    grid.z = (unsigned)(part == 1 ? 1 : split_last ? groups - 1 : groups);
    if constexpr (std::is_same<TA, float>::value && std::is_same<TC, float>::value) {
      RSVD_NB_SWITCH(nbv, {
        if (out_rowmajor) {
          if (vec)
            hipLaunchKernelGGL((tn_pipe_kernel<TP, TO, NB, true, true>), grid, dim3(256), 0, s, A, lda, K, N, P, ldp,
                               ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
          else
            hipLaunchKernelGGL((tn_pipe_kernel<TP, TO, NB, false, true>), grid, dim3(256), 0, s, A, lda, K, N, P, ldp,
                               ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
        } else {
          if (vec)
            hipLaunchKernelGGL((tn_pipe_kernel<TP, TO, NB, true, false>), grid, dim3(256), 0, s, A, lda, K, N, P, ldp,
                               ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
          else
            hipLaunchKernelGGL((tn_pipe_kernel<TP, TO, NB, false, false>), grid, dim3(256), 0, s, A, lda, K, N, P, ldp,
                               ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
        }
      });
    } else {
      RSVD_NB_SWITCH(nbv, {
        if (out_rowmajor) {
          if (vec)
            hipLaunchKernelGGL((tn_kernel<TA, TP, TC, TO, NB, true, true>), grid, dim3(256), 0, s, A, lda, K, N, P,
                               ldp, ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
          else
            hipLaunchKernelGGL((tn_kernel<TA, TP, TC, TO, NB, false, true>), grid, dim3(256), 0, s, A, lda, K, N, P,
                               ldp, ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
        } else {
          if (vec)
            hipLaunchKernelGGL((tn_kernel<TA, TP, TC, TO, NB, true, false>), grid, dim3(256), 0, s, A, lda, K, N, P,
                               ldp, ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
          else
            hipLaunchKernelGGL((tn_kernel<TA, TP, TC, TO, NB, false, false>), grid, dim3(256), 0, s, A, lda, K, N, P,
                               ldp, ncols, out, ldo, part_stride, kchunk, upper, out_skip, skip, cg_off);
        }
      });
    }
  }
  return hipGetLastError();
}

template <typename TA, typename TP, typename TC, typename TO>
hipError_t launch_tn(const TA* A, int64_t lda, int64_t K, int64_t N, const TP* P, int64_t ldp, int ncols, TO* out,
                     int64_t ldo, int64_t part_stride, int splits, bool out_rowmajor, hipStream_t s) {
  return launch_tn_k<TA, TP, TC, TO>(A, lda, K, N, P, ldp, ncols, out, ldo, part_stride, splits, out_rowmajor, false,
                                     s);
}

template <typename TP, typename TO>
hipError_t launch_reduce(const TP* part, int S, int64_t pstride, int64_t ldp, int64_t rows, int ncols, TO* out,
                         int64_t ldo, hipStream_t s, const int* skip) {
  int64_t work = ((rows + 3) / 4) * ncols;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL((reduce_kernel<TP, TO>), dim3((unsigned)((work + 255) / 256), 1), dim3(256), 0, s, part, S, S,
                     pstride, ldp, rows, ncols, out, ldo, (int64_t)0, skip);
  return hipGetLastError();
}

// Fixed-order sum of many partials: up to 2 group partials in one pass of reduce_kernel, more in one launch of
// reduce_tree_kernel (16 groups per entry; 196 partials of a 110 x 110 Gram: 5.7 us against two launches of
// 6.6 us for a two-level sum through tmp, which is no longer used).
template <typename TP>
hipError_t launch_reduce2(const TP* part, int S, int group, int64_t pstride, int64_t ldp, int64_t rows, int ncols,
                          TP* tmp, TP* out, int64_t ldo, hipStream_t s, const int* skip) {
  (void)tmp;
  if (S <= 2 * group) return launch_reduce<TP, TP>(part, S, pstride, ldp, rows, ncols, out, ldo, s, skip);
  const int64_t n = rows * ncols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((reduce_tree_kernel<TP>), dim3((unsigned)((n + 63) / 64)), dim3(1024), 0, s, part, S, pstride,
                     ldp, rows, ncols, out, ldo, skip);
  return hipGetLastError();
}

// out = A P for an upper-triangular P (the apply X <- X R^-1 of CholeskyQR): the triangular short-contraction
// kernel where it applies, otherwise the general product with each column group's contraction cut at its
// last column.
hipError_t launch_apply_upper(const float* A, int64_t lda, int64_t K, int64_t N, const float* P, int64_t ldp,
                              int ncols, float* out, int64_t ldo, hipStream_t s, const int* skip, float* out_skip) {
  return launch_tn_k<float, float, float, float>(A, lda, K, N, P, ldp, ncols, out, ldo, 0, 1, false, true, s, skip,
                                                 out_skip);
}

hipError_t launch_apply_upper(const float* A, int64_t lda, int64_t K, int64_t N, const double* P, int64_t ldp,
                              int ncols, double* out, int64_t ldo, hipStream_t s) {
  if (N <= 0 || ncols <= 0) return hipSuccess;
  if (K <= kApplyKMax && ncols <= kApplyKMax && K * lda < (int64_t(1) << 32) &&
      (int64_t)ncols * ldp < (int64_t(1) << 32))
    return launch_apply_small<double>(A, lda, (int)K, N, P, ldp, ncols, out, ldo, true, false, s);
  return launch_tn_k<float, double, double, double>(A, lda, K, N, P, ldp, ncols, out, ldo, 0, 1, false, true, s);
}

hipError_t launch_apply_upper(const double* A, int64_t lda, int64_t K, int64_t N, const double* P, int64_t ldp,
                              int ncols, double* out, int64_t ldo, hipStream_t s, const int* skip,
                              double* out_skip) {
  return launch_tn_k<double, double, double, double>(A, lda, K, N, P, ldp, ncols, out, ldo, 0, 1, false, true, s,
                                                     skip, out_skip);
}

// Explicit instantiations used by the host orchestration.
template hipError_t launch_nn<float, float, float, float>(const float*, int64_t, int64_t, int64_t, const float*,
                                                          int64_t, int, float*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_nn<double, double, double, double>(const double*, int64_t, int64_t, int64_t,
                                                              const double*, int64_t, int, double*, int64_t,
                                                              int64_t, int, hipStream_t);
template hipError_t launch_nn<float, float, double, double>(const float*, int64_t, int64_t, int64_t, const float*,
                                                            int64_t, int, double*, int64_t, int64_t, int,
                                                            hipStream_t);
template hipError_t launch_tn<float, float, float, float>(const float*, int64_t, int64_t, int64_t, const float*,
                                                          int64_t, int, float*, int64_t, int64_t, int, bool,
                                                          hipStream_t);
template hipError_t launch_tn<double, double, double, double>(const double*, int64_t, int64_t, int64_t,
                                                              const double*, int64_t, int, double*, int64_t,
                                                              int64_t, int, bool, hipStream_t);
template hipError_t launch_tn<float, double, double, double>(const float*, int64_t, int64_t, int64_t,
                                                             const double*, int64_t, int, double*, int64_t,
                                                             int64_t, int, bool, hipStream_t);
template hipError_t launch_reduce<float, float>(const float*, int, int64_t, int64_t, int64_t, int, float*, int64_t,
                                                hipStream_t, const int*);
template hipError_t launch_reduce<double, double>(const double*, int, int64_t, int64_t, int64_t, int, double*,
                                                  int64_t, hipStream_t, const int*);
template hipError_t launch_reduce2<double>(const double*, int, int, int64_t, int64_t, int64_t, int, double*, double*,
                                           int64_t, hipStream_t, const int*);

}  // namespace rsvd
