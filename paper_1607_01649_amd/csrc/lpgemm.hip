// Products of the low-precision copy of A with a thin FP32 panel, on MFMA with
// FP32 accumulation: out[split][c][r] = sum_{k in split} A(r, k) X(k, c).
//
//   bf16: v_mfma_f32_16x16x32_bf16, X rounded to bf16 (nearest even).
//   fp8:  v_mfma_f32_16x16x32_fp8_fp8 (OCP E4M3 on gfx950); A carries one
//         power-of-two scale per 128 x 128 tile, X one per 128-row segment of
//         each column, so a 128-wide contraction block is one tile column
//         and one segment: its partial product (four MFMAs into a fresh
//         accumulator) is added with the product of the two scales.
//
// The thin operand is converted once per product (panel_to_bf16 / _fp8) into
// a padded copy with 128-row segments, so the product kernel only moves bytes.
// A block of 256 threads owns 128 rows x 16 NB columns; a wave 32 rows (two
// 16-row MFMA blocks).  Each 128-wide contraction chunk: a lane loads 32
// contiguous values of each of its two rows (lane group g covers contraction
// indices 32 g .. 32 g + 31, fed to MFMA t as 32 g + 8 t + e on both
// operands), the X chunk is staged in LDS in fragment order.  The next
// chunk's A values and X fragments are loaded while the current one is
// multiplied (LDS double buffer, one barrier per chunk).
//
// Tile order: workgroups are dealt to the 8 XCDs round-robin by their linear
// index, so index L runs on XCD L % 8.  The column groups of one row block are
// given consecutive slots of one XCD (row block = 8 (slot / groups) + L % 8),
// so a tile of A fetched from HBM by the first of them is found in that XCD's
// L2 by the others.
#include "internal.hpp"
#include "lowp_common.hpp"

namespace rsvd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int LKC = 128;

// ------------------------------------------------------------------ thin-operand conversion

// Xq[c*ldq + k] = bf16(X[c*ldx + k]) for k < K, 0 for K <= k < ldq.  One thread per 8 values.
__global__ void panel_to_bf16_kernel(const float* __restrict__ X, int64_t ldx, int64_t K, int ncols,
                                     uint16_t* __restrict__ Xq, int64_t ldq) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per = ldq / 8;
  if (t >= per * ncols) return;
  const int64_t c = t / per, k = 8 * (t - c * per);
  uint16_t b[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) b[e] = (k + e < K) ? f32_to_bf16_rne(X[c * ldx + k + e]) : (uint16_t)0;
  *reinterpret_cast<uint4*>(Xq + c * ldq + k) =
      make_uint4(pack2(b[0], b[1]), pack2(b[2], b[3]), pack2(b[4], b[5]), pack2(b[6], b[7]));
}

// Xq[c*ldq + k] = E4M3(X / 2^e) with e per 128-row segment of column c (sX[c*(ldq/128) + seg] = 2^e).
// 16 consecutive threads cover one segment (amax by shuffles).
__global__ void panel_to_fp8_kernel(const float* __restrict__ X, int64_t ldx, int64_t K, int ncols,
                                    uint8_t* __restrict__ Xq, int64_t ldq, float* __restrict__ sX) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per = ldq / 8;
  const bool ok = t < per * ncols;
  const int64_t c = ok ? t / per : 0, k = ok ? 8 * (t - c * per) : 0;
  float v[8];
  float mx = 0.f;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    v[e] = (ok && k + e < K) ? X[c * ldx + k + e] : 0.f;
    mx = fmaxf(mx, fabsf(v[e]));
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 16));
  if (!ok) return;
  const int ex = fp8_scale_exp(mx);
  uint32_t w0 = 0, w1 = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    w0 |= f32_to_e4m3(ldexpf(v[e], -ex)) << (8 * e);
    w1 |= f32_to_e4m3(ldexpf(v[4 + e], -ex)) << (8 * e);
  }
  *reinterpret_cast<uint2*>(Xq + c * ldq + k) = make_uint2(w0, w1);
  if ((k & (LKC - 1)) == 0) sX[c * (ldq / LKC) + k / LKC] = ldexpf(1.0f, ex);
}

// ------------------------------------------------------------------ product

template <int KIND> struct LpFrag;   // 0: bf16, 1: fp8
template <> struct LpFrag<0> {
  typedef u32x4 X;                    // 8 bf16
  static constexpr int EB = 2;        // bytes per element
  static constexpr int AW = 4;        // 16-byte A loads per lane per row block per chunk
};
template <> struct LpFrag<1> {
  typedef u32x2 X;                    // 8 E4M3 codes
  static constexpr int EB = 1;
  static constexpr int AW = 2;
};

template <int KIND, int NB>
__global__ __launch_bounds__(256) void lp_nn_kernel(const uint8_t* __restrict__ A, int64_t lda,
                                                    const float* __restrict__ sA, int64_t s_row, int64_t s_k,
                                                    int64_t rows, int64_t K, const uint8_t* __restrict__ Xq,
                                                    int64_t ldq, const float* __restrict__ sX, int ncols, int groups,
                                                    int rblocks, float* __restrict__ out, int64_t ldo,
                                                    int64_t part_stride, int64_t kchunk) {
  typedef LpFrag<KIND> F;
  typedef typename F::X XF;
  constexpr int EB = F::EB, AW = F::AW;
  __shared__ XF xs[2][NB * 4 * 64];   // (buffer, cb, t, lane)
  __shared__ float sxs[2][NB * 16];
  typedef Mma<float> M;
  const int slot = blockIdx.x >> 3, xcd = blockIdx.x & 7;
  const int rb = (slot / groups) * 8 + xcd;
  const int cgi = slot - (slot / groups) * groups;
  if (rb >= rblocks) return;   // whole block: no barrier has been reached
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t rbase = (int64_t)rb * 128 + wave * 32;
  const int cg0 = cgi * NB * 16;
  const int split = blockIdx.y;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  const int64_t nseg = ldq / LKC;

  // staging assignment: slot u of this thread covers column cl(u), values 8 ch .. 8 ch + 7 of the chunk
  auto load_x = [&](int64_t k0, XF (&xr)[NB], float (&sr)[NB]) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = threadIdx.x + 256 * u;
      const int cl = it >> 4, ch = it & 15;
      const int c = cg0 + cl;
      if (c < ncols) {
        xr[u] = *reinterpret_cast<const XF*>(Xq + ((int64_t)c * ldq + k0 + 8 * ch) * EB);
        if constexpr (KIND == 1) sr[u] = sX[(int64_t)c * nseg + k0 / LKC];
      } else {
        xr[u] = XF{};
        sr[u] = 0.f;
      }
    }
  };
  auto store_x = [&](int buf, const XF (&xr)[NB], const float (&sr)[NB]) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int it = threadIdx.x + 256 * u;
      const int cl = it >> 4, ch = it & 15;
      const int cb = cl >> 4, cli = cl & 15, gg = ch >> 2, tt = ch & 3;
      xs[buf][(cb * 4 + tt) * 64 + cli + 16 * gg] = xr[u];
      if constexpr (KIND == 1)
        if (ch == 0) sxs[buf][cl] = sr[u];
    }
  };
  auto load_a = [&](int64_t k0, u32x4 (&ar)[2][AW]) {
#pragma unroll
    for (int rblk = 0; rblk < 2; ++rblk) {
      const int64_t r = rbase + 16 * rblk + li;
      if (r < rows) {
        const u32x4* p = reinterpret_cast<const u32x4*>(A + (r * lda + k0 + 32 * g) * EB);
#pragma unroll
        for (int w = 0; w < AW; ++w) ar[rblk][w] = p[w];
      } else {
#pragma unroll
        for (int w = 0; w < AW; ++w) ar[rblk][w] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  };

  f32x4 acc[2][NB];
#pragma unroll
  for (int rblk = 0; rblk < 2; ++rblk)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rblk][cb] = M::zero();

  XF xr[NB];
  float sr[NB];
  u32x4 ar[2][AW];
  if (kbeg < kend) {
    load_x(kbeg, xr, sr);
    load_a(kbeg, ar);
    store_x(0, xr, sr);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += LKC) {
    const bool more = k0 + LKC < kend;
    u32x4 an[2][AW];
    if (more) {
      load_x(k0 + LKC, xr, sr);
      load_a(k0 + LKC, an);
    }
    if constexpr (KIND == 0) {
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        bf16x8 b[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) b[cb] = __builtin_bit_cast(bf16x8, xs[cur][(cb * 4 + tt) * 64 + lane]);
#pragma unroll
        for (int rblk = 0; rblk < 2; ++rblk) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, ar[rblk][tt]);
#pragma unroll
          for (int cb = 0; cb < NB; ++cb)
            acc[rblk][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[cb], acc[rblk][cb], 0, 0, 0);
        }
      }
    } else {
      f32x4 part[2][NB];
#pragma unroll
      for (int rblk = 0; rblk < 2; ++rblk)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) part[rblk][cb] = M::zero();
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        long b[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) b[cb] = __builtin_bit_cast(long, xs[cur][(cb * 4 + tt) * 64 + lane]);
#pragma unroll
        for (int rblk = 0; rblk < 2; ++rblk) {
          const u32x4 q = ar[rblk][tt >> 1];
          const long av = (tt & 1) ? __builtin_bit_cast(long, u32x2{q[2], q[3]})
                                   : __builtin_bit_cast(long, u32x2{q[0], q[1]});
#pragma unroll
          for (int cb = 0; cb < NB; ++cb)
            part[rblk][cb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, b[cb], part[rblk][cb], 0, 0, 0);
        }
      }
      const float sa = sA[(int64_t)rb * s_row + (k0 / LKC) * s_k];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const float sc = sa * sxs[cur][cb * 16 + li];
#pragma unroll
        for (int rblk = 0; rblk < 2; ++rblk)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[rblk][cb][e] += sc * part[rblk][cb][e];
      }
    }
    if (more) store_x(cur ^ 1, xr, sr);
    __syncthreads();
    cur ^= 1;
    if (more) {
#pragma unroll
      for (int rblk = 0; rblk < 2; ++rblk)
#pragma unroll
        for (int w = 0; w < AW; ++w) ar[rblk][w] = an[rblk][w];
    }
  }

  float* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int rblk = 0; rblk < 2; ++rblk)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = cg0 + cb * 16 + li;
      if (c >= ncols) continue;
      const int64_t r = rbase + rblk * 16 + 4 * g;
      float* p = o + (int64_t)c * ldo + r;
      if (r + 4 <= rows) {
        *reinterpret_cast<float4*>(p) =
            make_float4(acc[rblk][cb][0], acc[rblk][cb][1], acc[rblk][cb][2], acc[rblk][cb][3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (r + e < rows) p[e] = acc[rblk][cb][e];
      }
    }
}

size_t lp_scratch_bytes(int kind, int64_t K, int ncols) {
  const size_t ldq = (size_t)((K + LKC - 1) / LKC) * LKC;
  const size_t codes = (size_t)ncols * ldq * (kind == 0 ? 2 : 1);
  const size_t scales = kind == 0 ? 0 : (size_t)ncols * (ldq / LKC) * sizeof(float);
  return (codes + 255) / 256 * 256 + scales;
}

int lp_splits_used(int64_t K, int splits) {
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + LKC - 1) / LKC * LKC;
  if (kchunk < LKC) kchunk = LKC;
  const int used = (int)((K + kchunk - 1) / kchunk);
  return used < 1 ? 1 : used;
}

// kind 0: A is bf16 (uint16 codes), 1: E4M3 codes with tile scales sA.  X is an FP32 panel (X[c*ldx + k]);
// scratch holds its converted copy (lp_scratch_bytes).
hipError_t launch_nn_lp(int kind, const void* A, int64_t lda, const float* sA, int64_t s_row, int64_t s_k,
                        int64_t rows, int64_t K, const float* X, int64_t ldx, int ncols, void* scratch, float* out,
                        int64_t ldo, int64_t part_stride, int splits, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (lda % LKC != 0 || lda < K || (reinterpret_cast<uintptr_t>(A) & 15) != 0 || !scratch ||
      (reinterpret_cast<uintptr_t>(scratch) & 255) != 0 || (kind == 1 && !sA))
    return hipErrorInvalidValue;
  const int64_t ldq = (K + LKC - 1) / LKC * LKC;
  uint8_t* Xq = reinterpret_cast<uint8_t*>(scratch);
  float* sX = kind == 1 ? reinterpret_cast<float*>(Xq + ((size_t)ncols * ldq + 255) / 256 * 256) : nullptr;
  const int64_t nthr = (ldq / 8) * ncols;
  if (kind == 0)
    hipLaunchKernelGGL(panel_to_bf16_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, X, ldx, K, ncols,
                       reinterpret_cast<uint16_t*>(Xq), ldq);
  else
    hipLaunchKernelGGL(panel_to_fp8_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, X, ldx, K, ncols,
                       Xq, ldq, sX);
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + LKC - 1) / LKC * LKC;
  if (kchunk < LKC) kchunk = LKC;
  const int used = (int)((K + kchunk - 1) / kchunk);
  // column tiles per block: capped where the accumulators would drop occupancy to one wave per SIMD
  const int nbmax = kind == 0 ? 7 : 5;
  int nb = (ncols + 15) / 16;
  nb = nb > nbmax ? nbmax : nb;
  const int groups = (ncols + nb * 16 - 1) / (nb * 16);
  const int rblocks = (int)((rows + 127) / 128);
  const int slots = (rblocks + 7) / 8 * groups;
  dim3 grid((unsigned)(slots * 8), (unsigned)used, 1);
  const uint8_t* Ab = reinterpret_cast<const uint8_t*>(A);
#define RSVD_LP_CASE(KV, NBV)                                                                                    \
  hipLaunchKernelGGL((lp_nn_kernel<KV, NBV>), grid, dim3(256), 0, s, Ab, lda, sA, s_row, s_k, rows, K, Xq, ldq, sX, \
                     ncols, groups, rblocks, out, ldo, part_stride, kchunk)
#define RSVD_LP_SWITCH(KV)                                                                                       \
  switch (nb) {                                                                                                  \
    case 1: RSVD_LP_CASE(KV, 1); break;                                                                          \
    case 2: RSVD_LP_CASE(KV, 2); break;                                                                          \
    case 3: RSVD_LP_CASE(KV, 3); break;                                                                          \
    case 4: RSVD_LP_CASE(KV, 4); break;                                                                          \
    case 5: RSVD_LP_CASE(KV, 5); break;                                                                          \
    case 6: RSVD_LP_CASE(KV, 6); break;                                                                          \
    case 7: RSVD_LP_CASE(KV, 7); break;                                                                          \
    default: RSVD_LP_CASE(KV, 8); break;                                                                         \
  }
  if (kind == 0) { RSVD_LP_SWITCH(0) } else { RSVD_LP_SWITCH(1) }
#undef RSVD_LP_SWITCH
#undef RSVD_LP_CASE
  return hipGetLastError();
}

}  // namespace rsvd
