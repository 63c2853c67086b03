// Gram matrix G = Y^T Y of a tall panel with FP64 accumulation (the first step
// of CholeskyQR, Section 2.3), on the FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// Y is an FP32 (or FP64) panel: column c contiguous, element (i, c) at
// Y[c*ld + i], K rows.  The output is the nc x nc matrix in the same partial
// layout as the other split products (out[split][c][r], a fixed-order sum
// over splits follows), so the reduction and the Cholesky that consume it do
// not change.
//
// G is symmetric: only the tile pairs (I, J), I <= J, of 128 x 128 tiles are
// computed, and each off-diagonal tile is written twice, as itself and
// transposed.  (Diagonal tiles of several-tile panels are computed whole:
// there every workgroup of the launch is resident at once, so a lighter diagonal workgroup would not
// shorten it.  A single tile, nc <= 128, has its own kernel below that computes only the 16 x 16
// blocks on and above the diagonal, dealt evenly to the waves.)  FP32 values are exact in FP64 and so are their products; the
// only rounding is the FP64 accumulation.
//
// Workgroup = 256 threads = 4 waves; tile pair from blockIdx.x, contraction
// range from blockIdx.y.  Wave w owns rows 32 w .. 32 w + 31 of tile I and all
// 128 columns of tile J.  Per chunk of KC rows of Y: the A operand (the wave's
// 32 columns of Y) is loaded straight into registers, 4 consecutive rows per
// lane (16-byte loads; the 16x16x4 MFMA consumes them over 4 instructions);
// the B operand (tile J's columns) is staged through LDS in fragment order,
// one linear 1 KB block per wave instruction.  The next chunk's loads are
// issued before the current chunk's products, all loads are unconditional
// (indices clamped, rows past K zeroed by a select), and the LDS hand-over
// uses a barrier without a vector-memory fence, so the loads stay in flight.
#include "internal.hpp"

namespace rsvd {

namespace {

template <typename TI> struct GramFmt;
template <> struct GramFmt<float> {
  typedef float4 V;
  static constexpr int KC = 64;
  static __device__ __forceinline__ double get(const V& v, int t) {
    return (double)(t == 0 ? v.x : t == 1 ? v.y : t == 2 ? v.z : v.w);
  }
};
template <> struct GramFmt<double> {
  struct V { double2 lo, hi; };
  static constexpr int KC = 32;   // half the rows: the staged chunk stays 32 KB
  static __device__ __forceinline__ double get(const V& v, int t) {
    return t == 0 ? v.lo.x : t == 1 ? v.lo.y : t == 2 ? v.hi.x : v.hi.y;
  }
};

template <typename TI>
__device__ __forceinline__ typename GramFmt<TI>::V gload4(const TI* p);
template <>
__device__ __forceinline__ GramFmt<float>::V gload4<float>(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}
template <>
__device__ __forceinline__ GramFmt<double>::V gload4<double>(const double* p) {
  GramFmt<double>::V v;
  v.lo = *reinterpret_cast<const double2*>(p);
  v.hi = *reinterpret_cast<const double2*>(p + 2);
  return v;
}

// Zero the entries whose row index k + t is >= K (only the last chunk of the panel has any).
template <typename V>
__device__ __forceinline__ V mask_rows(V v, int64_t k, int64_t K);
template <>
__device__ __forceinline__ float4 mask_rows<float4>(float4 v, int64_t k, int64_t K) {
  return make_float4(k < K ? v.x : 0.f, k + 1 < K ? v.y : 0.f, k + 2 < K ? v.z : 0.f, k + 3 < K ? v.w : 0.f);
}
template <>
__device__ __forceinline__ GramFmt<double>::V mask_rows<GramFmt<double>::V>(GramFmt<double>::V v, int64_t k,
                                                                            int64_t K) {
  v.lo.x = k < K ? v.lo.x : 0.0;
  v.lo.y = k + 1 < K ? v.lo.y : 0.0;
  v.hi.x = k + 2 < K ? v.hi.x : 0.0;
  v.hi.y = k + 3 < K ? v.hi.y : 0.0;
  return v;
}

__device__ __forceinline__ void lds_barrier_g() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((15) | (7 << 4) | (0 << 8) | (3 << 14));   // lgkmcnt(0) only
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

}  // namespace

template <typename TI, int NCB>
__global__ __launch_bounds__(256) void gram_kernel(const TI* __restrict__ Y, int64_t ld, int64_t K, int nc, int ntile,
                                                   int jfix, double* __restrict__ out, int64_t ldo,
                                                   int64_t part_stride, int64_t kchunk,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;   // a skipped second CholeskyQR pass (uniform: every thread reads the flag)
  typedef GramFmt<TI> F;
  typedef typename F::V V;
  constexpr int KC = F::KC;
  constexpr int NKQ = KC / 16;               // 16-row groups per chunk (4 MFMAs each)
  constexpr int NF = NCB * NKQ;              // fragment blocks of the staged B chunk
  constexpr int NFW = (NF + 3) / 4;          // per wave
  __shared__ V xs0[NF][64], xs1[NF][64];
  typedef Mma<double> M;

  // tile pair (I, J), I <= J: from the linear index over the upper triangle of ntile tiles, or (jfix >= 0) the
  // pair (blockIdx.x, jfix) of the last, partial column tile, whose NCB column blocks are only the live ones
  int I = 0, J = jfix;
  if (jfix >= 0) {
    I = blockIdx.x;
  } else {
    int rem = blockIdx.x;
    while (rem >= ntile - I) { rem -= ntile - I; ++I; }
    J = I + rem;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int split = blockIdx.y;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  const int64_t nck = (kend - kbeg + KC - 1) / KC;
  const int row0 = 128 * I + 32 * wave;      // first of this wave's 32 rows of G
  const int col0 = 128 * J;

  // operand addresses (clamped to real columns; padding columns are computed but never stored)
  const TI* pa[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) pa[rb] = Y + (int64_t)min(row0 + 16 * rb + M::arow(li), nc - 1) * ld + 4 * g;
  const TI* pb[NFW];
  int fbw[NFW];
#pragma unroll
  for (int u = 0; u < NFW; ++u) {
    const int fb = min(wave + 4 * u, NF - 1);   // waves past the last block repeat it (same data, same slot)
    fbw[u] = fb;
    const int cb = fb / NKQ, kq = fb - (fb / NKQ) * NKQ;
    pb[u] = Y + (int64_t)min(col0 + 16 * cb + li, nc - 1) * ld + 16 * kq + 4 * g;
  }

  auto kc = [&](int64_t i) { return kbeg + (i < nck ? i : nck - 1) * KC; };
  auto load = [&](int64_t k0, V (&a)[2][NKQ], V (&b)[NFW]) {
    const bool tail = k0 + KC > K;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int kq = 0; kq < NKQ; ++kq) {
        const int64_t k = k0 + 16 * kq + 4 * g;
        V v = gload4<TI>(pa[rb] + min(k0 + 16 * kq, ld - 16));
        a[rb][kq] = tail ? mask_rows(v, k, K) : v;
      }
#pragma unroll
    for (int u = 0; u < NFW; ++u) {
      const int kq = fbw[u] % NKQ;
      const int64_t k = k0 + 16 * kq + 4 * g;
      V v = gload4<TI>(pb[u] + min(k0, ld - KC));
      b[u] = tail ? mask_rows(v, k, K) : v;
    }
  };
  auto store_b = [&](const V (&b)[NFW], V (&xd)[NF][64]) {
#pragma unroll
    for (int u = 0; u < NFW; ++u) xd[fbw[u]][lane] = b[u];
  };

  typename M::acc acc[2][NCB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = M::zero();

  auto compute = [&](const V (&a)[2][NKQ], const V (&xb)[NF][64]) {
#pragma unroll
    for (int kq = 0; kq < NKQ; ++kq) {
      V b[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) b[cb] = xb[cb * NKQ + kq][lane];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const double av = F::get(a[rb][kq], t);
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = M::op(av, F::get(b[cb], t), acc[rb][cb]);
        }
    }
  };

  // step i: loads of chunk i+1 into the spare set, products of chunk i, its B into the other buffer, barrier
  V a0[2][NKQ], a1[2][NKQ], b0[NFW], b1[NFW];
  auto step = [&](int64_t i, const V (&acur)[2][NKQ], V (&anext)[2][NKQ], V (&bnext)[NFW], const V (&xc)[NF][64],
                  V (&xn)[NF][64]) {
    load(kc(i + 1), anext, bnext);
    __builtin_amdgcn_sched_barrier(0);
    compute(acur, xc);
    __builtin_amdgcn_sched_barrier(0);
    store_b(bnext, xn);
    lds_barrier_g();
  };
  load(kc(0), a0, b0);
  store_b(b0, xs0);
  lds_barrier_g();
  int64_t i = 0;
  for (; i + 2 <= nck; i += 2) {
    step(i, a0, a1, b1, xs0, xs1);
    step(i + 1, a1, a0, b0, xs1, xs0);
  }
  if (i < nck) step(i, a0, a1, b1, xs0, xs1);

  double* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = col0 + 16 * cb + li;
      const int r = row0 + 16 * rb + 4 * g;
      if (c >= nc) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (r + e < nc) {
          o[(int64_t)c * ldo + r + e] = acc[rb][cb][e];
          if (I != J) o[(int64_t)(r + e) * ldo + c] = acc[rb][cb][e];   // the mirror tile
        }
    }
}

// Single tile (nc <= 128): only the blocks on and above the diagonal, 28 of 49 for seven column blocks,
// dealt evenly to the waves (block b of the row-major upper triangle to wave b / PER).  The chunk's column
// blocks are all staged in LDS, one fragment per (column block, 16-row group) in the layout of the B
// operand, and the same fragment serves as the A operand: the FP64 MFMA then places column
// 16 rb + 4 e + g (not 16 rb + 4 g + e) in element e of lane group g, which the stores follow.
template <typename TI, int NCB>
__global__ __launch_bounds__(256) void gram_sym_kernel(const TI* __restrict__ Y, int64_t ld, int64_t K, int nc,
                                                       double* __restrict__ out, int64_t ldo, int64_t part_stride,
                                                       int64_t kchunk, const int* __restrict__ skip) {
  if (skip && *skip) return;   // a skipped second CholeskyQR pass (uniform: every thread reads the flag)
  typedef GramFmt<TI> F;
  typedef typename F::V V;
  constexpr int KC = F::KC;
  constexpr int NKQ = KC / 16;
  constexpr int NF = NCB * NKQ;
  constexpr int NFW = (NF + 3) / 4;
  constexpr int NBLK = NCB * (NCB + 1) / 2;
  constexpr int PER = (NBLK + 3) / 4;
  __shared__ V xs0[NF][64], xs1[NF][64];
  typedef Mma<double> M;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, li = lane & 15;
  const int split = blockIdx.y;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  const int64_t nck = (kend - kbeg + KC - 1) / KC;

  // staged fragment blocks (column block cb, row group kq): wave w moves blocks w, w + 4, ...
  const TI* pb[NFW];
  int fbw[NFW];
#pragma unroll
  for (int u = 0; u < NFW; ++u) {
    const int fb = min(wave + 4 * u, NF - 1);   // waves past the last block repeat it (same data, same slot)
    fbw[u] = fb;
    const int cb = fb / NKQ, kq = fb - (fb / NKQ) * NKQ;
    pb[u] = Y + (int64_t)min(16 * cb + li, nc - 1) * ld + 16 * kq + 4 * g;
  }
  // this wave's blocks (rb <= cb); a wave short of PER blocks repeats its last one and does not store it
  int rbj[PER], cbj[PER];
  bool okj[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    int b = wave * PER + j;
    okj[j] = b < NBLK;
    b = min(b, NBLK - 1);
    int rb = 0;
    while (b >= NCB - rb) { b -= NCB - rb; ++rb; }
    rbj[j] = rb;
    cbj[j] = rb + b;
  }

  auto kc = [&](int64_t i) { return kbeg + (i < nck ? i : nck - 1) * KC; };
  auto load = [&](int64_t k0, V (&b)[NFW]) {
    const bool tail = k0 + KC > K;
#pragma unroll
    for (int u = 0; u < NFW; ++u) {
      const int kq = fbw[u] % NKQ;
      const int64_t k = k0 + 16 * kq + 4 * g;
      V v = gload4<TI>(pb[u] + min(k0, ld - KC));
      b[u] = tail ? mask_rows(v, k, K) : v;
    }
  };
  auto store_b = [&](const V (&b)[NFW], V (&xd)[NF][64]) {
#pragma unroll
    for (int u = 0; u < NFW; ++u) xd[fbw[u]][lane] = b[u];
  };

  typename M::acc acc[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) acc[j] = M::zero();

  auto compute = [&](const V (&xb)[NF][64]) {
#pragma unroll
    for (int kq = 0; kq < NKQ; ++kq) {
      V a[PER], bb[PER];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        a[j] = xb[rbj[j] * NKQ + kq][lane];
        bb[j] = xb[cbj[j] * NKQ + kq][lane];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < PER; ++j) acc[j] = M::op(F::get(a[j], t), F::get(bb[j], t), acc[j]);
    }
  };

  V b0[NFW], b1[NFW];
  auto step = [&](int64_t i, V (&bnext)[NFW], const V (&xc)[NF][64], V (&xn)[NF][64]) {
    load(kc(i + 1), bnext);
    __builtin_amdgcn_sched_barrier(0);
    compute(xc);
    __builtin_amdgcn_sched_barrier(0);
    store_b(bnext, xn);
    lds_barrier_g();
  };
  load(kc(0), b0);
  store_b(b0, xs0);
  lds_barrier_g();
  int64_t i = 0;
  for (; i + 2 <= nck; i += 2) {
    step(i, b1, xs0, xs1);
    step(i + 1, b0, xs1, xs0);
  }
  if (i < nck) step(i, b1, xs0, xs1);

  double* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (!okj[j]) continue;
    const int rb = rbj[j], cb = cbj[j];
    const int c = 16 * cb + li;
    if (c >= nc) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * rb + 4 * e + g;
      if (r < nc) {
        o[(int64_t)c * ldo + r] = acc[j][e];
        if (rb != cb) o[(int64_t)r * ldo + c] = acc[j][e];   // the mirror block
      }
    }
  }
}

// Partials of G = Y^T Y (nc x nc, FP64) for `splits` contraction ranges of K rows; Y[c*ld + i] with ld >= K a
// multiple of 64 (so every chunk of rows lies inside the allocation), 16-byte aligned.  out[s*part_stride + c*ldo + r] for r, c < nc.  `splits` is
// a count normalised by nn_splits_used (ranges in multiples of 64 rows), so exactly `splits` partials are written.
template <typename TI>
hipError_t launch_gram(const TI* Y, int64_t ld, int64_t K, int nc, double* out, int64_t ldo, int64_t part_stride,
                       int splits, hipStream_t s, const int* skip) {
  if (nc <= 0 || K <= 0) return hipSuccess;
  if (ld < K || (ld % 64) != 0 || (reinterpret_cast<uintptr_t>(Y) & 15) != 0) return hipErrorInvalidValue;
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + 63) / 64 * 64;
  if (kchunk < 64) kchunk = 64;
  const int used = (int)((K + kchunk - 1) / kchunk);
  if (used != splits) return hipErrorInvalidValue;   // the consumer sums exactly `splits` partials
  const int ntile = (nc + 127) / 128;
  const int npair = ntile * (ntile + 1) / 2;
  int ncb = ntile == 1 ? (nc + 15) / 16 : 8;   // a single tile is as wide as the panel
  dim3 grid((unsigned)npair, (unsigned)used);
  int ntile_launch = ntile, jfix = -1;
#define RSVD_GRAM_CASE(N)                                                                                    \
  case N:                                                                                                  \
    hipLaunchKernelGGL((gram_kernel<TI, N>), grid, dim3(256), 0, s, Y, ld, K, nc, ntile_launch, jfix, out, ldo, \
                       part_stride, kchunk, skip);                                                         \
    break;
  if (ntile == 1) {
#define RSVD_GRAM_SYM_CASE(N)                                                                                    \
  case N:                                                                                                      \
    hipLaunchKernelGGL((gram_sym_kernel<TI, N>), grid, dim3(256), 0, s, Y, ld, K, nc, out, ldo, part_stride, kchunk, \
                       skip);                                                                                     \
    break;
    switch (ncb) {
      RSVD_GRAM_SYM_CASE(1)
      RSVD_GRAM_SYM_CASE(2)
      RSVD_GRAM_SYM_CASE(3)
      RSVD_GRAM_SYM_CASE(4)
      RSVD_GRAM_SYM_CASE(5)
      RSVD_GRAM_SYM_CASE(6)
      RSVD_GRAM_SYM_CASE(7)
      default: RSVD_GRAM_SYM_CASE(8)
    }
#undef RSVD_GRAM_SYM_CASE
    return hipGetLastError();
  }
  // A last tile with fewer than 8 live column blocks (ncb_last) is left out of the tile pairs of the full tiles,
  // which then take the same rows in more ranges (gram_tile_pairs counts only them), and its pairs (I, last)
  // go to a second launch with ncb_last column blocks: at 520 columns 10 full pairs and 5 pairs of one block
  // instead of 15 full pairs, 5 of them almost all padding.
  const int nfull = nc / 128;
  const int ncb_last = (nc - 128 * nfull + 15) / 16;
  const bool split_last = ntile > 1 && ncb_last > 0 && ncb_last < 8;
  for (int part = 0; part < (split_last ? 2 : 1); ++part) {
    if (split_last && part == 0) {
      ntile_launch = nfull;
      grid.x = (unsigned)(nfull * (nfull + 1) / 2);
    } else if (split_last) {
      ncb = ncb_last;
      jfix = nfull;
      grid.x = (unsigned)(nfull + 1);
    }
    switch (ncb) {
      RSVD_GRAM_CASE(1)
      RSVD_GRAM_CASE(2)
      RSVD_GRAM_CASE(3)
      RSVD_GRAM_CASE(4)
      RSVD_GRAM_CASE(5)
      RSVD_GRAM_CASE(6)
      RSVD_GRAM_CASE(7)
      default: RSVD_GRAM_CASE(8)
    }
  }
#undef RSVD_GRAM_CASE
  return hipGetLastError();
}

// Workgroups per contraction range of the Gram of an nc-column panel, for choosing the number of ranges: the
// pairs of full 128-column tiles (a partial last tile of fewer than 8 live column blocks goes to a short
// launch of its own).
int gram_tile_pairs(int nc) {
  const int ntile = (nc + 127) / 128;
  const int nfull = nc / 128;
  const int ncb_last = (nc - 128 * nfull + 15) / 16;
  if (ntile > 1 && ncb_last > 0 && ncb_last < 8) return nfull * (nfull + 1) / 2;
  return ntile * (ntile + 1) / 2;
}

template hipError_t launch_gram<float>(const float*, int64_t, int64_t, int, double*, int64_t, int64_t, int,
                                       hipStream_t, const int*);
template hipError_t launch_gram<double>(const double*, int64_t, int64_t, int, double*, int64_t, int64_t, int,
                                        hipStream_t, const int*);

}  // namespace rsvd
