// Products of the low-precision copy of A with a thin FP32 panel, on MFMA with
// FP32 accumulation: out[split][c][r] = sum_{k in split} A(r, k) X(k, c).
//
//   bf16: v_mfma_f32_16x16x32_bf16, X rounded to bf16 (nearest even).
//   fp8:  v_mfma_scale_f32_16x16x128_f8f6f4 on OCP E4M3 operands with the
//         block scales applied by the instruction: A carries one power-of-two
//         scale per 128 x 128 tile, X one per 128-row segment of each column,
//         so a 128-wide contraction chunk is one MFMA per 16 x 16 output tile
//         with the tile's scale on the A operand and the segment scales on the
//         B operand (both E8M0, exact for powers of two).
//
// The thin operand is converted once per product into a copy laid out in MFMA
// fragment order: for every 128-wide chunk and every 16 columns, the 1 KB
// blocks that one wave reads with a single 16-byte-per-lane load (4 blocks of
// 8 bf16 per lane, or 2 blocks of 16 E4M3 codes per lane).  Lane l of a block
// holds column l % 16 and the contraction indices 32 (l / 16) + 8 t + e (bf16,
// block t) or 32 (l / 16) + 16 h + e (fp8, block h); the A operand uses the
// same indices (a lane loads 32 contiguous values of its row), which is all
// the MFMA needs, whatever order it sums in.
//
// A block of 256 threads owns 256 rows x 16 NB columns, a wave 64 rows (four
// 16-row MFMA blocks), so each X fragment read from LDS feeds four MFMAs.
// Pipeline over pairs of chunks: the X fragments of the next pair and the A
// values one chunk ahead are loaded while the pair is multiplied, then the X
// fragments go to the spare of two LDS buffers (two chunks each); one barrier
// per pair, which leaves the A loads in flight (no fence: LDS completion is
// all it waits for).  Every load is unconditional (padded
// columns are zero, rows past the end are clamped and never stored, chunk
// indices past the end are clamped), so the compiler never has to wait for a
// load at a lane-masked join.
//
// A is read either row-major (the kernel-level entry points) or in the tiled layout of lowp_common.hpp (the
// library's own copies): there a workgroup's chunk is one contiguous block (64 KB bf16, 32 KB FP8) and each
// load instruction of a wave reads 1 KB contiguously, instead of 256-byte pieces of 256 rows; measured on
// 50000 x 20000 bf16, A X 448 -> 361 us and A^T Q 426 -> 348 us, identical results.
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
typedef int i32x8 __attribute__((ext_vector_type(8)));
constexpr int LKC = 128;          // contraction chunk (one FP8 scale block)
constexpr int LP_RB = 4;          // 16-row MFMA blocks per wave (a workgroup owns 64 LP_RB rows)
constexpr int LP_PD = 1;          // chunks of A loaded ahead

template <int KIND> struct LpFmt;
template <> struct LpFmt<0> {     // bf16
  static constexpr int EB = 2;    // bytes per element
  static constexpr int NFI = 4;   // 1 KB fragment blocks per 16 columns per chunk
  static constexpr int AW = 4;    // 16-byte A loads per lane per row block per chunk
};
template <> struct LpFmt<1> {     // E4M3
  static constexpr int EB = 1;
  static constexpr int NFI = 2;
  static constexpr int AW = 2;
};

// Column tiles of 16 per workgroup.  FP8 takes an even count so that the fragment blocks of a chunk split evenly
// over the four waves, at most 12: the fewest column groups (each re-reads A), then the fewest tiles per group
// (ncols = 520: three groups of 12 tiles, 576 columns, instead of five of 8, 640).
static int lp_nb(int kind, int ncols) {
  int nb = (ncols + 15) / 16;
  if (kind == 0) return nb > 7 ? 7 : nb;
  const int groups = (nb + 11) / 12;
  nb = (nb + groups - 1) / groups;
  return (nb + 1) & ~1;
}

// Columns of the converted panel: ncols rounded up to whole workgroups (non-decreasing in ncols).
static int lp_padded_cols(int kind, int ncols) {
  const int w = 16 * lp_nb(kind, ncols);
  return (ncols + w - 1) / w * w;
}

// ------------------------------------------------------------------ thin-operand conversion

// The 32 values X(col, kb .. kb+31) of one thread, zero past K and past ncols.  VEC (ldx and K multiples
// of 4, X 16-byte aligned): eight 16-byte loads at clamped addresses, each inside the first K entries of an
// existing column, then the out-of-range entries masked; otherwise guarded scalar loads (which the compiler
// waits for one at a time).
template <bool VEC>
__device__ __forceinline__ void load_seg32(const float* __restrict__ X, int64_t ldx, int64_t K, int ncols, int col,
                                           int64_t kb, float (&v)[32]) {
  if constexpr (VEC) {
    const float* base = X + (int64_t)min(col, ncols - 1) * ldx;
    float4 q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = *reinterpret_cast<const float4*>(base + min(kb + 4 * u, K - 4));
    const bool cok = col < ncols;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t k = kb + 4 * u;
      v[4 * u + 0] = (cok && k + 0 < K) ? q[u].x : 0.f;
      v[4 * u + 1] = (cok && k + 1 < K) ? q[u].y : 0.f;
      v[4 * u + 2] = (cok && k + 2 < K) ? q[u].z : 0.f;
      v[4 * u + 3] = (cok && k + 3 < K) ? q[u].w : 0.f;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      const int64_t k = kb + e;
      v[e] = (col < ncols && k < K) ? X[(int64_t)col * ldx + k] : 0.f;
    }
  }
}

// One thread per (chunk c, column block j, column cli, lane group gg): the 32 values X(col, k), col = 16 j + cli,
// k = 128 c + 32 gg + e, zero past K and past ncols.  bf16: four 16-byte pieces (e = 8 t ..) to block t.
template <bool VEC>
__global__ void panel_to_bf16_frag_kernel(const float* __restrict__ X, int64_t ldx, int64_t K, int ncols, int ncb,
                                          int64_t nthreads, uint8_t* __restrict__ Xf) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nthreads) return;
  const int gg = (int)(t & 3), cli = (int)((t >> 2) & 15);
  const int64_t rest = t >> 6, c = rest / ncb;
  const int j = (int)(rest - c * ncb);
  const int col = 16 * j + cli;
  const int64_t kb = c * LKC + 32 * gg;
  uint8_t* blk = Xf + (c * ncb + j) * (int64_t)(4 * 1024) + 16 * (cli + 16 * gg);
  float v[32];
  load_seg32<VEC>(X, ldx, K, ncols, col, kb, v);
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    uint16_t b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = f32_to_bf16_rne(v[8 * tt + e]);
    *reinterpret_cast<u32x4*>(blk + tt * 1024) =
        u32x4{pack2(b[0], b[1]), pack2(b[2], b[3]), pack2(b[4], b[5]), pack2(b[6], b[7])};
  }
}

// As above for E4M3: the four threads of a 128-row segment share its scale (amax by shuffles); two 16-byte
// pieces (e = 16 h ..) to block h; sXf[(c * ncb + j) * 16 + cli] = 2^e.
template <bool VEC>
__global__ void panel_to_fp8_frag_kernel(const float* __restrict__ X, int64_t ldx, int64_t K, int ncols, int ncb,
                                         int64_t nthreads, uint8_t* __restrict__ Xf, float* __restrict__ sXf) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool ok = t < nthreads;   // nthreads is a multiple of 64: whole waves agree
  const int gg = (int)(t & 3), cli = (int)((t >> 2) & 15);
  const int64_t rest = t >> 6, c = ok ? rest / ncb : 0;
  const int j = ok ? (int)(rest - c * ncb) : 0;
  const int col = 16 * j + cli;
  const int64_t kb = c * LKC + 32 * gg;
  float v[32];
  load_seg32<VEC>(X, ldx, K, ncols, ok ? col : ncols, kb, v);   // a thread past the end loads zeros
  float mx = 0.f;
#pragma unroll
  for (int e = 0; e < 32; ++e) mx = fmaxf(mx, fabsf(v[e]));
  mx = fmaxf(mx, __shfl_xor(mx, 1, 4));
  mx = fmaxf(mx, __shfl_xor(mx, 2, 4));
  if (!ok) return;
  const int ex = fp8_scale_exp(mx);
  uint8_t* blk = Xf + (c * ncb + j) * (int64_t)(2 * 1024) + 16 * (cli + 16 * gg);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float* vq = v + 16 * h + 4 * q;
      w[q] = f32x4_to_e4m3(ldexpf(vq[0], -ex), ldexpf(vq[1], -ex), ldexpf(vq[2], -ex), ldexpf(vq[3], -ex));
    }
    *reinterpret_cast<u32x4*>(blk + h * 1024) = u32x4{w[0], w[1], w[2], w[3]};
  }
  if (gg == 0) sXf[(c * ncb + j) * 16 + cli] = ldexpf(1.0f, ex);
}

// ------------------------------------------------------------------ product

// s_waitcnt with only the vector-memory count constrained (gfx9 encoding: vmcnt in bits 3:0 and 15:14).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier for LDS hand-over only: LDS operations complete first, vector-memory loads may stay in
// flight (the fence of __syncthreads would wait for them, which would end the prefetch at every chunk).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((15) | (7 << 4) | (0 << 8) | (3 << 14));   // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__device__ __forceinline__ i32x8 cat8(u32x4 a, u32x4 b) {
  return i32x8{(int)a[0], (int)a[1], (int)a[2], (int)a[3], (int)b[0], (int)b[1], (int)b[2], (int)b[3]};
}

// E8M0 code of a power of two held as a float (its biased exponent; 2^-127 is the subnormal with field 0).
__device__ __forceinline__ int e8m0_of(float s) { return (int)(__float_as_uint(s) >> 23); }

template <int KIND, int NB, int LRB, int PD, bool TILED>
__global__ __launch_bounds__(256) void lp_nn_kernel(const uint8_t* __restrict__ A, int64_t lda,
                                                    const float* __restrict__ sA, int64_t s_row, int64_t s_k,
                                                    int64_t rows, int64_t K, const uint8_t* __restrict__ Xf,
                                                    const float* __restrict__ sXf, int ncb, int ncols, int groups,
                                                    int rblocks, float* __restrict__ out, int64_t ldo,
                                                    int64_t part_stride, int64_t kchunk) {
  typedef LpFmt<KIND> F;
  constexpr int EB = F::EB, NFI = F::NFI, AW = F::AW;
  constexpr int LROWS = 64 * LRB;                     // rows per workgroup (LRB 16-row blocks per wave)
  constexpr int NF = NB * NFI;                        // fragment blocks per chunk
  static_assert(NF % 4 == 0, "fragment blocks must split evenly over the waves");
  constexpr int NXW = NF / 4;                         // fragment loads per wave per chunk
  // X fragments (and the fp8 scales of its columns), two buffers of two chunks: buffer b, chunk h of the pair
  __shared__ u32x4 xs[2][2][NF][64];
  __shared__ float sx[2][2][KIND == 1 ? 256 : 1];
  typedef Mma<float> M;
  const int slot = blockIdx.x >> 3, xcd = blockIdx.x & 7;
  const int rb = (slot / groups) * 8 + xcd;
  const int cgi = slot - (slot / groups) * groups;
  if (rb >= rblocks) return;   // whole workgroup: no barrier has been reached
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t rbase = (int64_t)rb * LROWS + wave * (16 * LRB);
  const int j0 = cgi * NB;
  const int split = blockIdx.y;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  const int64_t nck = (kend - kbeg + LKC - 1) / LKC;
  auto kc = [&](int64_t i) { return kbeg + (i < nck ? i : nck - 1) * LKC; };

  // X fragments (and fp8 scales) of the chunk at k0: wave w moves fragment blocks w, w + 4, ... (one linear
  // 16-byte load per lane from the fragment-ordered copy, one linear 16-byte LDS store).
  struct XStage {
    u32x4 v[NXW];
    float s;
  };
  // (Addresses are a workgroup-uniform base plus a 32-bit lane offset, which keeps them to one register each.)
  const uint32_t xoff = 16u * (uint32_t)(wave * 64 + lane);
  const uint32_t soff = 4u * (uint32_t)min(wave * 64 + lane, NB * 16 - 1);
  auto load_x = [&](int64_t k0, XStage& xr) {
    const int64_t c = k0 / LKC;
    const uint8_t* base = Xf + (c * ncb + j0) * (int64_t)(NFI * 1024);
#pragma unroll
    for (int f = 0; f < NXW; ++f) xr.v[f] = *reinterpret_cast<const u32x4*>(base + xoff + f * 4096u);
    if constexpr (KIND == 1)
      xr.s = *reinterpret_cast<const float*>(reinterpret_cast<const uint8_t*>(sXf + (c * ncb + j0) * 16) + soff);
    else
      xr.s = 0.f;
  };
  auto store_x = [&](const XStage& xr, u32x4 (&xd)[NF][64], float* sd) {
#pragma unroll
    for (int f = 0; f < NXW; ++f) xd[wave + 4 * f][lane] = xr.v[f];
    if constexpr (KIND == 1) sd[wave * 64 + lane] = xr.s;   // entries past the group are never read
  };
  static_assert(!TILED || (LRB == 4 && LROWS == kTileRows && LKC == kTileK), "tiled layout geometry");
  const int64_t row0 = (int64_t)rb * LROWS;
  // row-major: this workgroup's first row; tiled: its block of chunk 0 (rows past the end are zero there)
  const uint8_t* Ablk = TILED ? A + (int64_t)rb * (LROWS * LKC * EB) : A + row0 * lda * EB;
  uint32_t aoff[LRB];                         // < 256 rows x lda x EB (or one block): 32 bits suffice
#pragma unroll
  for (int rblk = 0; rblk < LRB; ++rblk) {
    if constexpr (TILED) {
      aoff[rblk] = (uint32_t)(((wave * LRB + rblk) * AW) * 1024 + lane * 16);
    } else {
      const int64_t r = min(rbase + 16 * rblk + li, rows - 1);   // rows past the end: a valid row, never stored
      aoff[rblk] = (uint32_t)(((r - row0) * lda + 32 * g) * EB);
    }
  }
  const int64_t cstride = (int64_t)rblocks * (LROWS * LKC * EB);   // tiled: bytes from one chunk's blocks to the next
  auto load_a = [&](int64_t k0, u32x4 (&ar)[LRB][AW]) {
    const uint8_t* base = TILED ? Ablk + (k0 / LKC) * cstride : Ablk + k0 * EB;
#pragma unroll
    for (int rblk = 0; rblk < LRB; ++rblk)
#pragma unroll
      for (int w = 0; w < AW; ++w)
        ar[rblk][w] = *reinterpret_cast<const u32x4*>(base + aoff[rblk] + (TILED ? 1024u : 16u) * w);
  };

  f32x4 acc[LRB][NB];
#pragma unroll
  for (int rblk = 0; rblk < LRB; ++rblk)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rblk][cb] = M::zero();

  auto compute = [&](const u32x4 (&xb)[NF][64], const float* sb_, const u32x4 (&ar)[LRB][AW], int64_t k0) {
    if constexpr (KIND == 0) {
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        bf16x8 b[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) b[cb] = __builtin_bit_cast(bf16x8, xb[cb * 4 + tt][lane]);
#pragma unroll
        for (int rblk = 0; rblk < LRB; ++rblk) {
          const bf16x8 av = __builtin_bit_cast(bf16x8, ar[rblk][tt]);
#pragma unroll
          for (int cb = 0; cb < NB; ++cb)
            acc[rblk][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[cb], acc[rblk][cb], 0, 0, 0);
        }
      }
    } else {
      // the wave's rows lie in one tile; a wave-uniform index makes this a scalar load.  A wave wholly past the
      // last row works on the clamped row rows - 1 (never stored), so it takes that row's tile: the index stays
      // inside the ceil(rows / 128) tile rows of the table.
      const int64_t trow = min(rbase, rows - 1) / 128;
      const int sidx = __builtin_amdgcn_readfirstlane((int)(trow * s_row + (k0 / LKC) * s_k));
      const int sa = e8m0_of(sA[sidx]);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const i32x8 bv = cat8(xb[2 * cb][lane], xb[2 * cb + 1][lane]);
        const int sb = e8m0_of(sb_[cb * 16 + li]);
#pragma unroll
        for (int rblk = 0; rblk < LRB; ++rblk) {
          const i32x8 av = cat8(ar[rblk][0], ar[rblk][1]);
          acc[rblk][cb] =
              __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc[rblk][cb], 0, 0, 0, sa, 0, sb);
        }
      }
    }
  };

  // Chunks are taken in pairs (i, i+1) from LDS buffer b: the loads of X for the next pair (i+2, i+3) and of
  // A(i+1) are issued, chunk i is multiplied, A(i+2) is issued, chunk i+1 is multiplied, then the next pair's
  // X goes to the other buffer and the workgroup passes one barrier (no fence: every global load stays in
  // flight) -- one barrier per two chunks.  A is one chunk ahead in registers, X two.  Register sets are
  // static (no copies); chunk indices past the end are clamped, so the last pair may repeat a chunk that is
  // never multiplied.
  static_assert(PD == 1, "one chunk of A ahead");
  XStage xp0, xp1;   // the next pair's X
  u32x4 a0[LRB][AW], a1[LRB][AW];
  load_x(kc(0), xp0);
  load_x(kc(1), xp1);
  load_a(kc(0), a0);
  store_x(xp0, xs[0][0], sx[0][0]);
  store_x(xp1, xs[0][1], sx[0][1]);
  lds_barrier();
  int64_t i = 0;
  int buf = 0;
  for (; i + 2 <= nck; i += 2) {
    load_x(kc(i + 2), xp0);
    load_x(kc(i + 3), xp1);
    load_a(kc(i + 1), a1);
    __builtin_amdgcn_sched_barrier(0);
    compute(xs[buf][0], sx[buf][0], a0, kc(i));
    __builtin_amdgcn_sched_barrier(0);
    load_a(kc(i + 2), a0);
    __builtin_amdgcn_sched_barrier(0);
    compute(xs[buf][1], sx[buf][1], a1, kc(i + 1));
    __builtin_amdgcn_sched_barrier(0);
    store_x(xp0, xs[buf ^ 1][0], sx[buf ^ 1][0]);
    store_x(xp1, xs[buf ^ 1][1], sx[buf ^ 1][1]);
    lds_barrier();
    buf ^= 1;
  }
  if (i < nck) compute(xs[buf][0], sx[buf][0], a0, kc(i));   // odd count: the last chunk, already staged

  float* o = out + (int64_t)split * part_stride;
#pragma unroll
  for (int rblk = 0; rblk < LRB; ++rblk)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = 16 * (j0 + cb) + li;
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

// Scratch: the fragment-ordered copy (nchunk x ncb blocks of NFI KB), then (fp8) its scales.
size_t lp_scratch_bytes(int kind, int64_t K, int ncols) {
  const size_t nchunk = (size_t)((K + LKC - 1) / LKC);
  const size_t ncb = (size_t)lp_padded_cols(kind, ncols) / 16;
  const size_t frag = nchunk * ncb * (kind == 0 ? 4096 : 2048);
  const size_t scales = kind == 0 ? 0 : nchunk * ncb * 16 * sizeof(float);
  return (frag + 255) / 256 * 256 + scales;
}

// Workgroups of a low-precision product along the row axis: row blocks of 64 * LP_RB rows,
// rounded up to whole XCD groups of 8, times the column groups.
int64_t lp_row_workgroups(int kind, int64_t rows, int ncols) {
  const int nb = lp_nb(kind, ncols);
  const int groups = lp_padded_cols(kind, ncols) / (nb * 16);
  const int64_t rblocks = (rows + 64 * LP_RB - 1) / (64 * LP_RB);
  return (rblocks + 7) / 8 * 8 * groups;
}

// Product workgroups resident at once on the current device: compute units x workgroups per
// unit (occupancy of the bf16 instantiation used at l <= 112); 256 if a query fails.
int lp_resident_workgroups() {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, cu = 0, per = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    cu = prop.multiProcessorCount;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, lp_nn_kernel<0, 7, LP_RB, LP_PD, true>, 256, 0) != hipSuccess)
    per = 0;
  cached = (cu > 0 && per > 0) ? cu * per : 256;
  return cached;
}

int lp_splits_used(int64_t K, int splits) {
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + LKC - 1) / LKC * LKC;
  if (kchunk < LKC) kchunk = LKC;
  const int used = (int)((K + kchunk - 1) / kchunk);
  return used < 1 ? 1 : used;
}

// kind 0: A is bf16 (uint16 codes), 1: E4M3 codes with tile scales sA.  X is an FP32 panel (X[c*ldx + k]);
// scratch holds its converted copy (lp_scratch_bytes).  tiled: A in the tiled layout of lowp_common.hpp (rows x
// K, lda unused), else row-major with leading dimension lda.
hipError_t launch_nn_lp(int kind, bool tiled, const void* A, int64_t lda, const float* sA, int64_t s_row,
                        int64_t s_k, int64_t rows, int64_t K, const float* X, int64_t ldx, int ncols, void* scratch,
                        float* out, int64_t ldo, int64_t part_stride, int splits, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (!tiled && (lda % LKC != 0 || lda < K)) return hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(A) & 15) != 0 || !scratch ||
      (reinterpret_cast<uintptr_t>(scratch) & 255) != 0 || (kind == 1 && !sA))
    return hipErrorInvalidValue;
  const int64_t nchunk = (K + LKC - 1) / LKC;
  const int nb = lp_nb(kind, ncols);
  const int cpad = lp_padded_cols(kind, ncols);
  const int ncb = cpad / 16;
  uint8_t* Xf = reinterpret_cast<uint8_t*>(scratch);
  const size_t frag = (size_t)nchunk * ncb * (kind == 0 ? 4096 : 2048);
  float* sXf = kind == 1 ? reinterpret_cast<float*>(Xf + (frag + 255) / 256 * 256) : nullptr;
  const int64_t nthr = nchunk * ncb * 64;
  const unsigned cgrid = (unsigned)((nthr + 255) / 256);
  const bool xvec = ldx % 4 == 0 && K % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  if (kind == 0) {
    if (xvec)
      hipLaunchKernelGGL(panel_to_bf16_frag_kernel<true>, dim3(cgrid), dim3(256), 0, s, X, ldx, K, ncols, ncb, nthr,
                         Xf);
    else
      hipLaunchKernelGGL(panel_to_bf16_frag_kernel<false>, dim3(cgrid), dim3(256), 0, s, X, ldx, K, ncols, ncb, nthr,
                         Xf);
  } else {
    if (xvec)
      hipLaunchKernelGGL(panel_to_fp8_frag_kernel<true>, dim3(cgrid), dim3(256), 0, s, X, ldx, K, ncols, ncb, nthr,
                         Xf, sXf);
    else
      hipLaunchKernelGGL(panel_to_fp8_frag_kernel<false>, dim3(cgrid), dim3(256), 0, s, X, ldx, K, ncols, ncb, nthr,
                         Xf, sXf);
  }
  if (splits < 1) splits = 1;
  int64_t kchunk = ((K + splits - 1) / splits + LKC - 1) / LKC * LKC;
  if (kchunk < LKC) kchunk = LKC;
  const int used = (int)((K + kchunk - 1) / kchunk);
  const int groups = cpad / (nb * 16);
  const int lrb = LP_RB;
  const int rblocks = (int)((rows + 64 * lrb - 1) / (64 * lrb));
  const int slots = (rblocks + 7) / 8 * groups;
  dim3 grid((unsigned)(slots * 8), (unsigned)used, 1);
  const uint8_t* Ab = reinterpret_cast<const uint8_t*>(A);
#define RSVD_LP_CASE(KV, NBV)                                                                                    \
  if (tiled)                                                                                                     \
    hipLaunchKernelGGL((lp_nn_kernel<KV, NBV, LP_RB, LP_PD, true>), grid, dim3(256), 0, s, Ab, lda, sA, s_row, s_k,   \
                       rows, K, Xf, sXf, ncb, ncols, groups, rblocks, out, ldo, part_stride, kchunk);               \
  else                                                                                                           \
    hipLaunchKernelGGL((lp_nn_kernel<KV, NBV, LP_RB, LP_PD, false>), grid, dim3(256), 0, s, Ab, lda, sA, s_row, s_k,  \
                       rows, K, Xf, sXf, ncb, ncols, groups, rblocks, out, ldo, part_stride, kchunk)
  if (kind == 0) {
    switch (nb) {
      case 1: RSVD_LP_CASE(0, 1); break;
      case 2: RSVD_LP_CASE(0, 2); break;
      case 3: RSVD_LP_CASE(0, 3); break;
      case 4: RSVD_LP_CASE(0, 4); break;
      case 5: RSVD_LP_CASE(0, 5); break;
      case 6: RSVD_LP_CASE(0, 6); break;
      default: RSVD_LP_CASE(0, 7); break;
    }
  } else {
    switch (nb) {
      case 2: RSVD_LP_CASE(1, 2); break;
      case 4: RSVD_LP_CASE(1, 4); break;
      case 6: RSVD_LP_CASE(1, 6); break;
      case 8: RSVD_LP_CASE(1, 8); break;
      case 10: RSVD_LP_CASE(1, 10); break;
      default: RSVD_LP_CASE(1, 12); break;
    }
  }
#undef RSVD_LP_CASE
  return hipGetLastError();
}

}  // namespace rsvd
