// Host runtime behind the C ABI of include/rsvd.h: argument validation,
// workspace carving, split selection and the launch sequence of the
// randomized SVD (Figure 5 of the paper plus Stage B of Section 3).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/rsvd.h"
#include "internal.hpp"

using namespace rsvd;

namespace {

constexpr int kRedGroup = 16;   // partials summed per first-level reduction group
constexpr int kSkipFlag = 16;   // flags word: the current orthonormalisation may skip its second pass
// Column-scaled condition bound below which an intermediate basis takes one CholeskyQR pass: orthogonal to
// about 1e6 u in FP64 and 1e3 u in the FP32 panel product, ample for a basis that is multiplied again.
constexpr double kOrthSkipKappa = 1e3;
// device status words: [0] non-finite pivot, [1] dropped columns, [2] Jacobi
// not converged, [3] Jacobi sweeps, [4] non-finite entry of A (conversion),
// [8] and [9] non-finite and dropped pivots of the Nystrom core factor B2 = C^T C
constexpr int kFlags = 64;
// selector: grid of oversampling values (power steps 0 .. kSelNQ-1), and floats of selector scratch
// (network input 16, hidden activations 64 + 64, logits 40)
constexpr int kSelNP = 8, kSelNQ = 5;
constexpr int kSelP[kSelNP] = {0, 5, 10, 20, 40, 80, 160, 320};
constexpr int kSelFloats = 16 + 64 + 64 + 40;

bool log_enabled() {
  static int v = -1;
  if (v < 0) v = getenv("RSVD_LOG") ? 1 : 0;
  return v == 1;
}

#define RSVD_LOGF(...)                        \
  do {                                        \
    if (log_enabled()) {                      \
      fprintf(stderr, "[rsvd] " __VA_ARGS__); \
      fputc('\n', stderr);                    \
    }                                         \
  } while (0)

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Byte offsets of the workspace regions (all 256-byte aligned).
struct Layout {
  int l, LP;          // sketch width k+p and its 16-multiple
  int lmax, LPmax;    // capacity of Q and B^T (max_rank when certifying), and its 16-multiple
  int b, bw;          // fallback block and its 16-multiple
  int r;              // certificate probes
  int W;              // width of the sketch-side panels: max(LP, bw)
  int64_t ldm, ldn;
  size_t es;   // element size of panels (8 for F64, 4 otherwise)
  int s_nn, s_tn, s_gm, s_gn, s_nn16, s_tn16;
  int64_t ld16, ldT;   // leading dimensions of the bf16 copies of A and A^T
  size_t a16, a16t, a8, a8t, s8, xq, omega, gc, Y, T, Q, Z, Wp, Bt, agc, E, tmpr, zr, tmpn, small, small2, part, gpart, gpart2, G, R1, R, rinv,
      rinv_d, Q1d, sigma, uhat_d, uhat_p, vhat_p, scr_chol, scr_jac, norms, frob, flags, sel, srht_sgn, srht_sub,
      gr, sp, cp_S, cp_nrm, cp_orig, cp_bmax, cp_bidx, cp_cnt, cp_Q, cp_J, cp_Z, cp_small, total;
  int64_t ldS;   // leading dimension of the pivoted QR's S (rows of length max(m, n))
};

int pick_splits(int64_t tiles, int64_t K, int64_t target, int64_t min_chunk) {
  int64_t s = (target + tiles - 1) / std::max<int64_t>(tiles, 1);
  int64_t cap = std::max<int64_t>(1, K / min_chunk);
  s = std::min(std::max<int64_t>(s, 1), cap);
  return (int)std::min<int64_t>(s, 1024);
}

// Split count of a low-precision product: as many contraction ranges as fit in one wave of
// the resident workgroups (at least one).  The products stream A once; one wave of long
// workgroups beats several waves of short ones, and each extra range writes one more
// partial panel that the reduction reads back (at l = 110 on 50000 x 20000 the former
// choice of ~2048 workgroups wrote 0.24 GB of partials per A^T product).
int lp_pick_splits(int64_t row_wgs, int64_t K, int resident) {
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(64, K / 512));
  return (int)std::min<int64_t>(cap, std::max<int64_t>(1, resident / std::max<int64_t>(row_wgs, 1)));
}

// Contraction ranges of the Gram (multiples of 64 rows) so that pairs x ranges <= 256 workgroups, as many as fit.
int gram_splits(int pairs, int64_t K) {
  const int64_t nchunk = (K + 63) / 64;
  const int64_t target = std::max<int64_t>(1, 256 / std::max(pairs, 1));
  const int64_t per = (nchunk + target - 1) / target;   // chunks per range
  return (int)std::max<int64_t>(1, (nchunk + per - 1) / per);
}

bool validate(const rsvd_desc* d) {
  if (!d) return false;
  if (d->m < 1 || d->n < 1 || d->k < 1) return false;
  const bool sel = d->p == -1 && d->q == -1;
  if (!sel && (d->p < 0 || d->q < 0)) return false;
  int64_t l = (int64_t)d->k + (sel ? 0 : d->p);
  if (l > std::min(d->m, d->n) || l > 1024) return false;
  if (d->a_dtype != RSVD_F64 && d->a_dtype != RSVD_F32) return false;
  if (!(d->eps >= 0.0) || !isfinite(d->eps)) return false;
  if (d->n_probe < 0 || d->n_probe > 64 || d->est_power < 0 || d->est_power > 8) return false;
  if (d->fallback_block < 0 || d->fallback_block > 256 || d->max_rank < 0) return false;
  if (d->max_rank > 0 && d->max_rank < l) return false;
  if (d->max_rank > std::min<int64_t>(std::min(d->m, d->n), 1024)) return false;
  if (d->m > (int64_t)1 << 40 || d->n > (int64_t)1 << 40) return false;
  if (d->flags & RSVD_NYSTROM) {
    if (sel || d->m != d->n || d->eps != 0.0) return false;
  }
  if (const uint32_t spf = d->flags & (RSVD_SINGLE_PASS | RSVD_SINGLE_PASS_SYM)) {
    if (spf == (RSVD_SINGLE_PASS | RSVD_SINGLE_PASS_SYM)) return false;
    if (sel || d->q != 0 || d->eps != 0.0 || d->sketch_dtype != d->proj_dtype) return false;
    if (d->sketch_dtype != d->a_dtype && d->sketch_dtype != RSVD_BF16) return false;
    if (d->flags & (RSVD_RETURN_RANK_L | RSVD_SKETCH_SRHT | RSVD_NYSTROM)) return false;
    if ((spf & RSVD_SINGLE_PASS_SYM) && d->m != d->n) return false;
  }
  if (d->flags & RSVD_ID_CUR) {
    if (sel || d->eps != 0.0 || d->sketch_dtype != d->a_dtype || d->proj_dtype != d->a_dtype) return false;
    if (l > cpqr_max_rows()) return false;
    if (d->flags & (RSVD_RETURN_RANK_L | RSVD_SKETCH_SRHT | RSVD_NYSTROM | RSVD_SINGLE_PASS | RSVD_SINGLE_PASS_SYM))
      return false;
  }
  if (d->flags & RSVD_SKETCH_SRHT) {
    if (sel || d->sketch_dtype != d->a_dtype) return false;
    if (d->n > srht_max_n(d->a_dtype == RSVD_F64 ? 8 : 4)) return false;
  }
  return true;
}

bool uses_bf16(const rsvd_desc* d) { return d->sketch_dtype == RSVD_BF16 || d->proj_dtype == RSVD_BF16; }
bool uses_fp8(const rsvd_desc* d) { return d->sketch_dtype == RSVD_FP8_E4M3 || d->proj_dtype == RSVD_FP8_E4M3; }

rsvd_status supported(const rsvd_desc* d) {
  if (d->a_dtype == RSVD_F64) {
    if (d->sketch_dtype != RSVD_F64 || d->proj_dtype != RSVD_F64) return RSVD_E_UNSUPPORTED;
  } else {
    auto ok = [](int t) { return t == RSVD_F32 || t == RSVD_BF16 || t == RSVD_FP8_E4M3; };
    if (!ok(d->sketch_dtype) || !ok(d->proj_dtype)) return RSVD_E_UNSUPPORTED;
  }
  return RSVD_OK;
}

Layout make_layout(const rsvd_desc* d) {
  Layout L{};
  const bool cert = d->eps > 0.0;
  L.l = d->k + d->p;
  L.LP = (int)round_up(L.l, 16);
  L.lmax = cert ? std::max(L.l, (int)d->max_rank) : L.l;
  L.LPmax = (int)round_up(L.lmax, 16);
  L.b = cert ? (d->fallback_block ? d->fallback_block : 32) : 0;
  L.bw = (int)round_up(L.b, 16);
  L.r = cert ? (d->n_probe ? d->n_probe : 10) : 0;
  L.W = std::max({L.LP, L.bw, (int)round_up(std::max(L.r, 1), 16)});
  L.ldm = round_up(d->m, 64);
  L.ldn = round_up(d->n, 64);
  L.es = (d->a_dtype == RSVD_F64) ? 8 : 4;
  const int64_t cg = (L.l + 127) / 128;
  L.s_nn = pick_splits(((d->m + 127) / 128) * cg, d->n, 2048, 512);
  L.s_tn = pick_splits(((d->n + 255) / 256) * cg, d->m, 2048, 512);
  // Gram: one workgroup per CU (it needs the whole register file), so aim for at most 256 workgroups
  const int gp = gram_tile_pairs(L.l);
  L.s_gm = gram_splits(gp, d->m);
  L.s_gn = gram_splits(gp, d->n);
  L.s_nn = nn_splits_used(d->n, L.s_nn);
  L.s_tn = nn_splits_used(d->m, L.s_tn);
  L.s_gm = nn_splits_used(d->m, L.s_gm);
  L.s_gn = nn_splits_used(d->n, L.s_gn);
  {
    const int kind_nn = d->sketch_dtype == RSVD_FP8_E4M3 ? 1 : 0;   // Y = A X products
    const int kind_tn = d->proj_dtype == RSVD_FP8_E4M3 ? 1 : 0;     // A^T Q products
    const int res = lp_resident_workgroups();
    L.s_nn16 = lp_splits_used(d->n, lp_pick_splits(lp_row_workgroups(kind_nn, d->m, L.l), d->n, res));
    L.s_tn16 = lp_splits_used(d->m, lp_pick_splits(lp_row_workgroups(kind_tn, d->n, L.l), d->m, res));
  }
  L.ld16 = round_up(d->n, 128);
  L.ldT = round_up(d->m, 128);
  const size_t LP = (size_t)L.LP, LPM = (size_t)L.LPmax, Wd = (size_t)L.W;
  const size_t R = (size_t)std::max(L.r, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = round_up(off + bytes, 256); return o; };
  const bool b16 = uses_bf16(d);
  // the low-precision copies are in the tiled layout (rows padded to 256, contraction to 128)
  L.a16 = take(b16 ? bf16_tiled_bytes(d->m, d->n) : 256);
  L.a16t = take(b16 ? bf16_tiled_bytes(d->n, d->m) : 256);
  const bool b8 = uses_fp8(d);
  L.a8 = take(b8 ? fp8_tiled_bytes(d->m, d->n) : 256);
  L.a8t = take(b8 ? fp8_tiled_bytes(d->n, d->m) : 256);
  L.s8 = take(b8 ? (size_t)(L.ld16 / 128) * (L.ldT / 128) * sizeof(float) : 256);
  // converted thin operand of a low-precision product (widest panel, longest contraction)
  L.xq = take((b16 || b8) ? lp_scratch_bytes(b16 ? 0 : 1, std::max(d->m, d->n), std::max({L.W, L.LPmax, 16})) : 256);
  L.omega = take(Wd * L.ldn * L.es);
  L.gc = take(R * L.ldn * L.es);
  L.Y = take(Wd * L.ldm * L.es);
  L.T = take(std::max(Wd, LPM) * std::max(L.ldm, L.ldn) * L.es);
  L.Q = take(LPM * L.ldm * L.es);
  L.Z = take(LP * L.ldn * L.es);
  L.Wp = take(LP * L.ldn * L.es);
  L.Bt = take(LPM * L.ldn * L.es);
  L.agc = take(R * L.ldm * L.es);
  L.E = take(R * L.ldm * L.es);
  L.tmpr = take(std::max(R, (size_t)L.bw) * L.ldm * L.es);
  L.zr = take(R * L.ldn * L.es);
  L.tmpn = take(R * L.ldn * L.es);
  L.small = take(LPM * std::max(LPM, R) * 8);
  L.small2 = take(LPM * std::max(LPM, R) * 8);
  const size_t sa = std::max({(size_t)L.s_nn, (size_t)L.s_nn16}), sb = std::max({(size_t)L.s_tn, (size_t)L.s_tn16});
  L.part = take(std::max(sa * Wd * L.ldm, sb * Wd * L.ldn) * L.es);
  const size_t sg = (size_t)std::max(L.s_gm, L.s_gn);
  L.gpart = take(sg * LPM * std::max(LPM, R) * 8);
  L.gpart2 = take(((sg + kRedGroup - 1) / kRedGroup) * LPM * LPM * 8);
  L.G = take(LPM * LPM * 8);
  L.R1 = take(LPM * LPM * 8);
  L.R = take(LPM * LPM * 8);
  L.rinv = take(LPM * LPM * L.es);
  L.rinv_d = take(LPM * LPM * 8);
  const bool single_pass = (d->flags & (RSVD_SINGLE_PASS | RSVD_SINGLE_PASS_SYM)) != 0;
  L.Q1d = take(LPM * (single_pass ? std::max(L.ldm, L.ldn) : L.ldn) * 8);
  L.sigma = take(LPM * 8);
  L.uhat_d = take(LPM * LPM * 8);
  L.uhat_p = take(LPM * LPM * L.es);
  L.vhat_p = take(LPM * LPM * L.es);
  L.scr_chol = take(LPM > 128 ? chol_blocked_scratch_doubles((int)LPM) * 8 : 256);
  L.scr_jac = take(LPM > 128 ? jacobi_blocked_scratch_bytes((int)LPM) : 256);
  L.norms = take(64 * 8);
  L.frob = take(1040 * 8);
  L.flags = take(kFlags * sizeof(int));
  L.sel = take(kSelFloats * sizeof(float));
  const bool srht = (d->flags & RSVD_SKETCH_SRHT) != 0;
  L.srht_sgn = take(srht ? (size_t)d->n * L.es : 256);
  L.srht_sub = take(srht ? 1024 * sizeof(int) : 256);
  // single pass: the row-space test matrix G_r (m x l panel) and the FP64 k x k core (13 LP x LP matrices)
  L.gr = take((d->flags & RSVD_SINGLE_PASS) ? Wd * L.ldm * L.es : 256);
  L.sp = take(single_pass ? 13 * LP * LP * 8 : 256);
  // interpolative decompositions: the pivoted QR's S (k rows of length max(m, n)), norms, block maxima, q vectors,
  // pivots (two sets), CUR's Z (k x n) and its k x k matrices
  const bool idc = (d->flags & RSVD_ID_CUR) != 0;
  const int64_t nmax = std::max(d->m, d->n);
  L.ldS = round_up(nmax, 64);
  const size_t nbk = idc ? (size_t)cpqr_blocks(nmax) : 1;
  L.cp_S = take(idc ? (size_t)d->k * L.ldS * 8 : 256);
  L.cp_nrm = take(idc ? (size_t)nmax * 8 : 256);
  L.cp_orig = take(idc ? (size_t)nmax * 8 : 256);
  L.cp_bmax = take(nbk * 8);
  L.cp_bidx = take(nbk * sizeof(int));
  L.cp_cnt = take(sizeof(unsigned));
  L.cp_Q = take(idc ? LP * LP * 8 : 256);
  L.cp_J = take(idc ? 2 * LP * sizeof(int) : 256);
  L.cp_Z = take(idc ? (size_t)d->k * L.ldn * 8 : 256);
  L.cp_small = take(idc ? 6 * LP * LP * 8 : 256);
  L.total = off;
  return L;
}

// Selector mode (p = q = -1): the layouts of every grid point fit in the workspace; this returns the largest.
bool selector_mode(const rsvd_desc* d) { return d->p == -1 && d->q == -1; }

int sel_lcap(const rsvd_desc* d) { return (int)std::min<int64_t>({d->m, d->n, (int64_t)1024}); }

rsvd_desc derived_desc(const rsvd_desc* d, int p, int q) {
  rsvd_desc e = *d;
  e.p = p;
  e.q = q;
  if (e.max_rank > 0 && e.max_rank < e.k + p) e.max_rank = e.k + p;
  return e;
}

Layout make_layout_any(const rsvd_desc* d) {
  if (!selector_mode(d)) return make_layout(d);
  Layout best{};
  bool have = false;
  for (int ip = 0; ip < kSelNP; ++ip) {
    if (d->k + kSelP[ip] > sel_lcap(d)) continue;
    rsvd_desc e = derived_desc(d, kSelP[ip], kSelNQ - 1);
    Layout L = make_layout(&e);
    if (!have || L.total > best.total) best = L;
    have = true;
  }
  return best;
}

}  // namespace

struct rsvd_plan_s {
  rsvd_desc d;
  Layout L;
  hipStream_t st;
  char* ws;
  int device;
  bool timing;
  hipEvent_t ev[8];
  static constexpr int kGemmEv = 256;          // event pairs around A-products (RSVD_TIMING)
  hipEvent_t gev[2 * kGemmEv];
  int gkind[kGemmEv];                          // 0 = A*X, 1 = A^T*X
  int ngemm = 0;
  // selector parameters (selector mode)
  const float* theta = nullptr;
  float tau = 0.5f;
  int p_used = 0, q_used = 0;
  // results of the last call (host side)
  int rank_out = 0, fallback_steps = 0;
  double err_bound = 0.0, frob_res = -1.0;
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      RSVD_LOGF("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return RSVD_E_HIP;                                                     \
    }                                                                        \
  } while (0)

#define RS_TRY(expr)                        \
  do {                                      \
    rsvd_status s_ = (expr);                \
    if (s_ != RSVD_OK) return s_;           \
  } while (0)

inline int lp16(int nc) { return (int)round_up(nc, 16); }

template <typename T> struct Path {
  rsvd_plan_s& P;
  const Layout& L;
  hipStream_t st;
  double tau;
  explicit Path(rsvd_plan_s& p) : P(p), L(p.L), st(p.st) {
    const double u = sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
    tau = (double)L.lmax * u * u;
  }

  void mark(int i) { if (P.timing) (void)hipEventRecord(P.ev[i], st); }
  int gemm_begin(int kind) {
    if (!P.timing || P.ngemm >= rsvd_plan_s::kGemmEv) return -1;
    int i = P.ngemm++;
    P.gkind[i] = kind;
    (void)hipEventRecord(P.gev[2 * i], st);
    return i;
  }
  void gemm_end(int i) { if (i >= 0) (void)hipEventRecord(P.gev[2 * i + 1], st); }

  // G (nc x nc, column-major, ld lp16(nc)) = X^T X for a nc-column panel X with `rows` rows, FP64 accumulation.
  // With `skip`, both launches return at once when *skip is set (a skipped second CholeskyQR pass).
  rsvd_status gram(const T* X, int64_t ldx, int64_t rows, int nc, int splits, double* G, const int* skip = nullptr) {
    const int LPc = lp16(nc);
    double* gp = P.at<double>(L.gpart);
    HIP_TRY(launch_gram<T>(X, ldx, rows, nc, gp, LPc, (int64_t)LPc * LPc, splits, st, skip));
    HIP_TRY(launch_reduce2<double>(gp, splits, kRedGroup, (int64_t)LPc * LPc, LPc, nc, nc, P.at<double>(L.gpart2), G,
                                   LPc, st, skip));
    return RSVD_OK;
  }

  // out = X R^-1 (R^-1 upper triangular, nc x nc at leading dimension LPc).
  // With `skip`, a set *skip on the device sends the product to out_skip instead of out (nowhere when
  // out_skip is null).
  hipError_t apply_rinv(const T* X, int64_t ld, int64_t rows, int nc, const T* rinv, int LPc, T* out,
                        const int* skip = nullptr, T* out_skip = nullptr) {
    return launch_apply_upper(X, ld, nc, rows, rinv, LPc, nc, out, ld, st, skip, out_skip);
  }

  // out = orth(X) for an nc-column panel: CholeskyQR2 (two passes of G = X^T X = R^T R, X <- X R^-1).
  // may_skip (a basis that is multiplied again, not the one Stage B uses): the second pass is
  // skipped on the device when the first pass's factor bounds the column-scaled condition number of X by
  // kOrthSkipKappa (the first apply then writes `out`, which must not alias X, and the second pass's Gram, sum,
  // Cholesky and apply return at once), since one pass
  // then leaves a basis orthonormal to about kappa^2 u plus kappa times the panel's rounding.
  rsvd_status orth(const T* X, int64_t ld, int64_t rows, int nc, int splits, T* out, bool may_skip = false) {
    const int LPc = lp16(nc);
    double* G = P.at<double>(L.G);
    T* rinv = P.at<T>(L.rinv);
    T* tmp = P.at<T>(L.T);
    int* flags = P.at<int>(L.flags);
    double* scr = P.at<double>(L.scr_chol);
    int* skip = (may_skip && out != X) ? flags + kSkipFlag : nullptr;
    RS_TRY(gram(X, ld, rows, nc, splits, G));
    HIP_TRY(launch_chol<T>(G, LPc, nc, LPc, tau, rinv, nullptr, nullptr, scr, flags, st, skip, kOrthSkipKappa));
    HIP_TRY(apply_rinv(X, ld, rows, nc, rinv, LPc, tmp, skip, out));   // skipped: this is the basis
    RS_TRY(gram(tmp, ld, rows, nc, splits, G, skip));
    HIP_TRY(launch_chol<T>(G, LPc, nc, LPc, tau, rinv, nullptr, nullptr, scr, flags, st, nullptr, 0.0, skip));
    HIP_TRY(apply_rinv(tmp, ld, rows, nc, rinv, LPc, out, skip));      // skipped: nothing to do
    return RSVD_OK;
  }

  // Y = A X (m x nc panel) for an n-row panel X, operands in precision `dt`.
  rsvd_status apply_a(const T* A, int64_t lda, const T* X, int nc, T* Y, int dt) {
    T* part = P.at<T>(L.part);
    const int64_t m = P.d.m, n = P.d.n;
    const int LPc = lp16(nc);
    int S = L.s_nn;
    int ev = gemm_begin(0);
    if (dt == RSVD_BF16) {
      if constexpr (sizeof(T) == 4) {
        S = L.s_nn16;
        HIP_TRY(launch_nn_lp(0, true, P.at<uint16_t>(L.a16), L.ld16, nullptr, 0, 0, m, n, X, L.ldn, nc, P.at<char>(L.xq),
                             S == 1 ? Y : part, L.ldm, (int64_t)LPc * L.ldm, S, st));
      }
    } else if (dt == RSVD_FP8_E4M3) {
      if constexpr (sizeof(T) == 4) {
        S = L.s_nn16;
        HIP_TRY(launch_nn_lp(1, true, P.at<uint8_t>(L.a8), L.ld16, P.at<float>(L.s8), L.ld16 / 128, 1, m, n, X, L.ldn, nc,
                             P.at<char>(L.xq), S == 1 ? Y : part, L.ldm, (int64_t)LPc * L.ldm, S, st));
      }
    } else {
      HIP_TRY((launch_nn<T, T, T, T>(A, lda, m, n, X, L.ldn, nc, part, L.ldm, (int64_t)LPc * L.ldm, S, st)));
    }
    gemm_end(ev);
    const bool direct = S == 1 && (dt == RSVD_BF16 || dt == RSVD_FP8_E4M3) && sizeof(T) == 4;   // written in place
    if (!direct) HIP_TRY((launch_reduce<T, T>(part, S, (int64_t)LPc * L.ldm, L.ldm, m, nc, Y, L.ldm, st)));
    return RSVD_OK;
  }

  // Z = A^T Q (n x nc panel) for an m-row panel Q, operands in precision `dt`.
  rsvd_status apply_at(const T* A, int64_t lda, const T* Qp, int nc, T* Z, int dt) {
    T* part = P.at<T>(L.part);
    const int64_t m = P.d.m, n = P.d.n;
    const int LPc = lp16(nc);
    int S = L.s_tn;
    int ev = gemm_begin(1);
    if (dt == RSVD_BF16) {
      if constexpr (sizeof(T) == 4) {
        S = L.s_tn16;
        HIP_TRY(launch_nn_lp(0, true, P.at<uint16_t>(L.a16t), L.ldT, nullptr, 0, 0, n, m, Qp, L.ldm, nc, P.at<char>(L.xq),
                             S == 1 ? Z : part, L.ldn, (int64_t)LPc * L.ldn, S, st));
      }
    } else if (dt == RSVD_FP8_E4M3) {
      if constexpr (sizeof(T) == 4) {
        S = L.s_tn16;
        HIP_TRY(launch_nn_lp(1, true, P.at<uint8_t>(L.a8t), L.ldT, P.at<float>(L.s8), 1, L.ld16 / 128, n, m, Qp, L.ldm, nc,
                             P.at<char>(L.xq), S == 1 ? Z : part, L.ldn, (int64_t)LPc * L.ldn, S, st));
      }
    } else {
      HIP_TRY(
          (launch_tn<T, T, T, T>(A, lda, m, n, Qp, L.ldm, nc, part, L.ldn, (int64_t)LPc * L.ldn, S, false, st)));
    }
    gemm_end(ev);
    const bool direct = S == 1 && (dt == RSVD_BF16 || dt == RSVD_FP8_E4M3) && sizeof(T) == 4;   // written in place
    if (!direct) HIP_TRY((launch_reduce<T, T>(part, S, (int64_t)LPc * L.ldn, L.ldn, n, nc, Z, L.ldn, st)));
    return RSVD_OK;
  }

  // C (na x nb, stored C[j*ldc + i] = (Xa^T Xb)(i, j)) for panels Xa (na columns) and Xb (nb columns) of `rows`
  // rows; split over the rows, summed in fixed order.
  rsvd_status panel_tprod(const T* Xa, int na, const T* Xb, int nb, int64_t ld, int64_t rows, int splits, T* C,
                          int64_t ldc) {
    T* gp = P.at<T>(L.gpart);
    HIP_TRY((launch_nn<T, T, T, T>(Xa, ld, na, rows, Xb, ld, nb, gp, ldc, (int64_t)ldc * nb, splits, st)));
    HIP_TRY((launch_reduce<T, T>(gp, splits, (int64_t)ldc * nb, ldc, na, nb, C, ldc, st)));
    return RSVD_OK;
  }

  // out (rows x nb panel) = X S for an na-column panel X and S (na x nb, S[j*lds + i]).
  rsvd_status panel_mult(const T* X, int na, int64_t ld, int64_t rows, const T* S, int64_t lds, int nb, T* out,
                         int64_t ldo) {
    HIP_TRY((launch_tn<T, T, T, T>(X, ld, na, rows, S, lds, nb, out, ldo, 0, 1, false, st)));
    return RSVD_OK;
  }

  // SVD of B (nc x n, held as the panel B^T): FP64 CholeskyQR2 of B^T, Jacobi on R^T.
  rsvd_status small_svd(int nc) { return small_svd_panel(P.at<T>(L.Bt), L.ldn, P.d.n, nc, L.s_gn); }

  // The same for any nc-column panel X (rows x nc, leading dimension ld) in place of B^T: leaves sigma, U_hat
  // (uhat_d, uhat_p) and vhat_p = U_hat diag(sigma)^-1, so that X vhat_p holds X's left singular vectors.
  rsvd_status small_svd_panel(const T* X, int64_t ld, int64_t rows, int nc, int splits) {
    const int LPc = lp16(nc);
    double* G = P.at<double>(L.G);
    double* R1 = P.at<double>(L.R1);
    double* R = P.at<double>(L.R);
    double* rinv_d = P.at<double>(L.rinv_d);
    double* Q1d = P.at<double>(L.Q1d);
    double* gp = P.at<double>(L.gpart);
    double* gp2 = P.at<double>(L.gpart2);
    double* scr = P.at<double>(L.scr_chol);
    int* flags = P.at<int>(L.flags);
    HIP_TRY(launch_gram<T>(X, ld, rows, nc, gp, LPc, (int64_t)LPc * LPc, splits, st));
    HIP_TRY(launch_reduce2<double>(gp, splits, kRedGroup, (int64_t)LPc * LPc, LPc, nc, nc, gp2, G, LPc, st));
    HIP_TRY(launch_chol<double>(G, LPc, nc, LPc, tau, rinv_d, R1, nullptr, scr, flags, st));
    HIP_TRY(launch_apply_upper(X, ld, nc, rows, rinv_d, LPc, nc, Q1d, ld, st));   // R1^-1 upper triangular
    HIP_TRY(launch_gram<double>(Q1d, ld, rows, nc, gp, LPc, (int64_t)LPc * LPc, splits, st));
    HIP_TRY(launch_reduce2<double>(gp, splits, kRedGroup, (int64_t)LPc * LPc, LPc, nc, nc, gp2, G, LPc, st));
    HIP_TRY(launch_chol<double>(G, LPc, nc, LPc, tau, rinv_d, R, R1, scr, flags, st));
    // Jacobi stops when every pair's cosine is below tol: l u for FP64 data; for FP32 data (whose own
    // rounding is 6e-8) 1e-10 already leaves U_hat orthogonal and sigma exact far below that, and saves
    // about one sweep.
    const double tol = std::max((double)nc * 2.220446049250313e-16, sizeof(T) == 4 ? 1e-10 : 0.0);
    HIP_TRY(launch_jacobi<T>(R, nc, LPc, tol, 60, P.at<double>(L.sigma), P.at<double>(L.uhat_d), P.at<T>(L.uhat_p),
                             P.at<T>(L.vhat_p), P.at<double>(L.scr_jac), flags, st));
    return RSVD_OK;
  }

  // U = Q U_hat(:, :kout), V = B^T U_hat D^-1 (:, :kout), S = sigma(:kout) for a basis of nc columns.
  rsvd_status lift(int nc, int kout, T* U, int64_t ldu, double* S, T* V, int64_t ldv) {
    const int64_t m = P.d.m, n = P.d.n;
    const int LPc = lp16(nc);
    HIP_TRY((launch_tn<T, T, T, T>(P.at<T>(L.Q), L.ldm, nc, m, P.at<T>(L.uhat_p), LPc, kout, U, ldu, 0, 1, true, st)));
    if (V)
      HIP_TRY((launch_tn<T, T, T, T>(P.at<T>(L.Bt), L.ldn, nc, n, P.at<T>(L.vhat_p), LPc, kout, V, ldv, 0, 1, true,
                                     st)));
    HIP_TRY(hipMemcpyAsync(S, P.at<double>(L.sigma), (size_t)kout * sizeof(double), hipMemcpyDeviceToDevice, st));
    return RSVD_OK;
  }

  // H (nc x r, ld LPmax) <- U_hat_k U_hat_k^T H, the projector onto the k kept directions of the small SVD.
  rsvd_status apply_pk(int nc, int kk, T* H) {
    const int LPc = lp16(nc);
    T* W1 = P.at<T>(L.small2);
    HIP_TRY((launch_nn<T, T, T, T>(P.at<T>(L.uhat_p), LPc, kk, nc, H, L.LPmax, L.r, W1, L.LPmax, 0, 1, st)));
    HIP_TRY((launch_tn<T, T, T, T>(P.at<T>(L.uhat_p), LPc, kk, nc, W1, L.LPmax, L.r, H, L.LPmax, 0, 1, false, st)));
    return RSVD_OK;
  }

  rsvd_status max_colnorm(const T* E, double* h_max) {
    double* nrm = P.at<double>(L.norms);
    HIP_TRY(launch_colnorm<T>(E, L.ldm, P.d.m, L.r, nrm, st));
    double h[64];
    HIP_TRY(hipMemcpyAsync(h, nrm, (size_t)L.r * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double mx = 0.0;
    for (int i = 0; i < L.r; ++i) mx = std::max(mx, h[i]);
    *h_max = mx;
    return RSVD_OK;
  }

  // Certificate (Section 14 with the Lemma of Section 13).  T = A - Q P B with P = U_hat_k U_hat_k^T (the
  // rank-k result, kk > 0) or P = I (the rank-nc pair (Q, B), kk == 0); U D V^T = Q P B for the factors the
  // library returns.  E = (T T^T)^s T Gc is left in the E panel; returns max_i ||E(:, i)||.
  rsvd_status cert_residual(const T* A, int64_t lda, int nc, int kk, double* h_max) {
    const int64_t m = P.d.m, n = P.d.n;
    const int r = L.r;
    const int dt = (sizeof(T) == 8) ? RSVD_F64 : RSVD_F32;   // the certificate judges A itself
    T* E = P.at<T>(L.E);
    T* H = P.at<T>(L.small);
    T* tmp = P.at<T>(L.tmpr);
    T* Zr = P.at<T>(L.zr);
    T* tn_ = P.at<T>(L.tmpn);
    T* Q = P.at<T>(L.Q);
    T* Bt = P.at<T>(L.Bt);
    // E = A Gc - Q P (B Gc)
    HIP_TRY(hipMemcpyAsync(E, P.at<T>(L.agc), (size_t)r * L.ldm * sizeof(T), hipMemcpyDeviceToDevice, st));
    RS_TRY(panel_tprod(Bt, nc, P.at<T>(L.gc), r, L.ldn, n, L.s_gn, H, L.LPmax));
    if (kk > 0) RS_TRY(apply_pk(nc, kk, H));
    RS_TRY(panel_mult(Q, nc, L.ldm, m, H, L.LPmax, r, tmp, L.ldm));
    HIP_TRY(launch_axpy_panel<T>(E, L.ldm, tmp, L.ldm, m, r, T(-1), st));
    for (int t = 0; t < P.d.est_power; ++t) {
      // Zr = T^T E = A^T E - B^T P (Q^T E)
      RS_TRY(apply_at(A, lda, E, r, Zr, dt));
      RS_TRY(panel_tprod(Q, nc, E, r, L.ldm, m, L.s_gm, H, L.LPmax));
      if (kk > 0) RS_TRY(apply_pk(nc, kk, H));
      RS_TRY(panel_mult(Bt, nc, L.ldn, n, H, L.LPmax, r, tn_, L.ldn));
      HIP_TRY(launch_axpy_panel<T>(Zr, L.ldn, tn_, L.ldn, n, r, T(-1), st));
      // E = T Zr = A Zr - Q P (B Zr)
      RS_TRY(apply_a(A, lda, Zr, r, E, dt));
      RS_TRY(panel_tprod(Bt, nc, Zr, r, L.ldn, n, L.s_gn, H, L.LPmax));
      if (kk > 0) RS_TRY(apply_pk(nc, kk, H));
      RS_TRY(panel_mult(Q, nc, L.ldm, m, H, L.LPmax, r, tmp, L.ldm));
      HIP_TRY(launch_axpy_panel<T>(E, L.ldm, tmp, L.ldm, m, r, T(-1), st));
    }
    return max_colnorm(E, h_max);
  }

  double bound_from(double mx) const {
    const double c_alpha = 10.0 * sqrt(2.0 / 3.14159265358979323846);   // (1/alpha) sqrt(2/pi), alpha = 1/10
    const int s = P.d.est_power;
    return pow(c_alpha * mx, 1.0 / (2 * s + 1));
  }

  // Low-precision copies of A (bf16, or FP8 with tile scales) for the formats the description asks for; the
  // scan for non-finite entries of A is counted in flags[4].
  rsvd_status prep_lowp(const T* A, int64_t lda) {
    const int64_t m = P.d.m, n = P.d.n;
    int* flags = P.at<int>(L.flags);
    if (uses_bf16(&P.d)) {
      if constexpr (sizeof(T) == 4)
        HIP_TRY(launch_to_bf16_tiled(A, lda, m, n, P.at<uint16_t>(L.a16), P.at<uint16_t>(L.a16t), flags + 4, st));
    }
    if (uses_fp8(&P.d)) {
      if constexpr (sizeof(T) == 4)
        HIP_TRY(launch_to_fp8_tiled(A, lda, m, n, P.at<uint8_t>(L.a8), P.at<uint8_t>(L.a8t), P.at<float>(L.s8),
                                    flags + 4, st));
    }
    return RSVD_OK;
  }

  // Stage A (Figure 5): input preparation, Omega, Q = orth(A Omega) and q power steps with
  // re-orthonormalisation after every application of A or A^T; leaves Q (m x l panel).
  rsvd_status stage_a(const T* A, int64_t lda, const double* omega_in) {
    const int64_t m = P.d.m, n = P.d.n;
    const int l = L.l;
    T* omega = P.at<T>(L.omega);
    T* Y = P.at<T>(L.Y);
    T* Q = P.at<T>(L.Q);
    T* Z = P.at<T>(L.Z);
    T* Wp = P.at<T>(L.Wp);
    int* flags = P.at<int>(L.flags);
    const int sk = P.d.sketch_dtype;
    RS_TRY(prep_lowp(A, lda));
    if ((P.d.flags & RSVD_SKETCH_SRHT) && !omega_in) {
      // Section 6: Y = A Omega with the structured test matrix, one pass over A.
      T* sgn = P.at<T>(L.srht_sgn);
      int* sub = P.at<int>(L.srht_sub);
      HIP_TRY(launch_srht_setup<T>(P.d.seed, (int)n, l, sgn, sub, st));
      int ev = gemm_begin(0);
      HIP_TRY(launch_srht_sketch<T>(A, lda, m, (int)n, sgn, sub, l, Y, 1, L.ldm, st));
      gemm_end(ev);
    } else {
      // Figure 5 (1): Gaussian test matrix.
      if (omega_in)
        HIP_TRY(launch_rowmajor_to_panel<T>(omega_in, n, l, l, omega, L.ldn, st));
      else
        HIP_TRY(launch_gaussian<T>(P.d.seed, 4u, n, l, 0, omega, 1, L.ldn, st));
      RS_TRY(apply_a(A, lda, omega, l, Y, sk));
    }
    // (2): Q = orth(A Omega).  Every basis but the last is multiplied again (the second CholeskyQR pass may
    // be skipped there).
    RS_TRY(orth(Y, L.ldm, m, l, L.s_gm, Q, P.d.q > 0));
    mark(1);
    // (3)-(6): q power steps with re-orthonormalisation.
    for (int it = 0; it < P.d.q; ++it) {
      RS_TRY(apply_at(A, lda, Q, l, Z, sk));
      RS_TRY(orth(Z, L.ldn, n, l, L.s_gn, Wp, true));
      RS_TRY(apply_a(A, lda, Wp, l, Y, sk));
      RS_TRY(orth(Y, L.ldm, m, l, L.s_gm, Q, it + 1 < P.d.q));
    }
    mark(2);
    return RSVD_OK;
  }

  // Selector probe: sigma(A G16) with 16 Gaussian columns of stream 5 (FP64 CholeskyQR of the Gram and
  // Jacobi, as for the small SVD) into L.sigma[0..16); the network input into the selector scratch.
  rsvd_status probe(const T* A, int64_t lda) {
    const int64_t m = P.d.m, n = P.d.n;
    T* omega = P.at<T>(L.omega);
    T* Y = P.at<T>(L.Y);
    double* G = P.at<double>(L.G);
    double* R = P.at<double>(L.R);
    int* flags = P.at<int>(L.flags);
    const int dt = (sizeof(T) == 8) ? RSVD_F64 : RSVD_F32;
    HIP_TRY(launch_gaussian<T>(P.d.seed, 5u, n, 16, 0, omega, 1, L.ldn, st));
    RS_TRY(apply_a(A, lda, omega, 16, Y, dt));
    RS_TRY(gram(Y, L.ldm, m, 16, L.s_gm, G));
    HIP_TRY(launch_chol<double>(G, 16, 16, 16, tau, P.at<double>(L.rinv_d), R, nullptr, P.at<double>(L.scr_chol), flags,
                                st));
    HIP_TRY(launch_jacobi<T>(R, 16, 16, 16 * 2.220446049250313e-16, 60, P.at<double>(L.sigma), P.at<double>(L.uhat_d),
                             (T*)nullptr, (T*)nullptr, P.at<double>(L.scr_jac), flags, st));
    HIP_TRY(launch_sel_features(P.at<double>(L.sigma), P.d.k, P.at<float>(L.sel), st));
    return RSVD_OK;
  }

  // Certificates of the prefixes Q_w of the Stage A basis (see rsvd_prefix_bounds).
  rsvd_status prefix_bounds(const T* A, int64_t lda, int nw, const int* widths, double* bounds) {
    const int64_t m = P.d.m, n = P.d.n;
    const int r = L.r;
    int* flags = P.at<int>(L.flags);
    HIP_TRY(launch_fill_int(flags, kFlags, 0, st));
    RS_TRY(stage_a(A, lda, nullptr));
    T* gc = P.at<T>(L.gc);
    T* agc = P.at<T>(L.agc);
    T* E = P.at<T>(L.E);
    T* H = P.at<T>(L.small);
    T* tmp = P.at<T>(L.tmpr);
    T* Q = P.at<T>(L.Q);
    const int dt = (sizeof(T) == 8) ? RSVD_F64 : RSVD_F32;
    HIP_TRY(launch_gaussian<T>(P.d.seed, 6u, n, r, 0, gc, 1, L.ldn, st));
    RS_TRY(apply_a(A, lda, gc, r, agc, dt));
    for (int i = 0; i < nw; ++i) {
      const int w = widths[i];
      HIP_TRY(hipMemcpyAsync(E, agc, (size_t)r * L.ldm * sizeof(T), hipMemcpyDeviceToDevice, st));
      RS_TRY(panel_tprod(Q, w, agc, r, L.ldm, m, L.s_gm, H, L.LPmax));
      RS_TRY(panel_mult(Q, w, L.ldm, m, H, L.LPmax, r, tmp, L.ldm));
      HIP_TRY(launch_axpy_panel<T>(E, L.ldm, tmp, L.ldm, m, r, T(-1), st));
      double mx = 0.0;
      RS_TRY(max_colnorm(E, &mx));
      bounds[i] = bound_from(mx);
    }
    return RSVD_OK;
  }

  // Section 9: the Nystrom eigendecomposition of a symmetric positive semidefinite A (m == n).
  rsvd_status run_nystrom(const T* A, int64_t lda, const double* omega_in, T* U, int64_t ldu, double* S, T* V,
                          int64_t ldv, int kout) {
    const int64_t n = P.d.n;
    const int l = L.l, LPc = lp16(l);
    int* flags = P.at<int>(L.flags);
    P.rank_out = kout;
    P.fallback_steps = 0;
    P.err_bound = 0.0;
    P.frob_res = -1.0;
    mark(0);
    HIP_TRY(launch_fill_int(flags, kFlags, 0, st));
    RS_TRY(stage_a(A, lda, omega_in));   // steps 1-3: Q (n x l panel)
    T* Q = P.at<T>(L.Q);
    T* B1 = P.at<T>(L.T);
    T* Bt = P.at<T>(L.Bt);
    RS_TRY(apply_a(A, lda, Q, l, B1, P.d.proj_dtype));   // step 4: B1 = A Q
    mark(3);
    // B2 = Q^T B1 with FP64 accumulation, made exactly symmetric
    double* G = P.at<double>(L.G);
    double* gp = P.at<double>(L.gpart);
    HIP_TRY((launch_nn<T, T, double, double>(Q, L.ldm, l, n, B1, L.ldm, l, gp, LPc, (int64_t)LPc * LPc, L.s_gm,
                                             st)));
    HIP_TRY((launch_reduce<double, double>(gp, L.s_gm, (int64_t)LPc * LPc, LPc, l, l, G, LPc, st)));
    HIP_TRY(launch_symmetrize(G, LPc, l, st));
    // step 5: B2 = C^T C; B2 is the Gram matrix of A^(1/2) Q, accurate to u relative to its diagonal, so
    // a pivot at or below l u of it is dependent and dropped (counted apart from the CholeskyQR steps)
    const double u = sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
    HIP_TRY(launch_chol<T>(G, LPc, l, LPc, (double)l * u, P.at<T>(L.rinv), nullptr, nullptr, P.at<double>(L.scr_chol),
                           flags + 8, st));
    // step 6: F = B1 C^-1, into the B^T panel (m == n: the two panels share their leading dimension)
    HIP_TRY(apply_rinv(B1, L.ldm, n, l, P.at<T>(L.rinv), LPc, Bt));
    // step 7: SVD of F, as the SVD of F^T held as its panel F: F^T = U_hat Sigma W^T
    RS_TRY(small_svd(l));
    mark(4);
    // U = F U_hat Sigma^-1 (the left singular vectors of F), S = Sigma^2 (step 8), V = U
    HIP_TRY((launch_tn<T, T, T, T>(Bt, L.ldn, l, n, P.at<T>(L.vhat_p), LPc, kout, U, ldu, 0, 1, true, st)));
    if (V)
      HIP_TRY((launch_tn<T, T, T, T>(Bt, L.ldn, l, n, P.at<T>(L.vhat_p), LPc, kout, V, ldv, 0, 1, true, st)));
    HIP_TRY(launch_square(P.at<double>(L.sigma), S, kout, st));
    mark(5);
    return RSVD_OK;
  }

  // C (na x nb, FP64, C[j*ldc + i] = (Xa^T Xb)(i, j)) for panels Xa, Xb of `rows` rows, FP64 accumulation, split
  // over the rows and summed in fixed order.
  rsvd_status tprod64(const T* Xa, int na, const T* Xb, int nb, int64_t ld, int64_t rows, int splits, double* C,
                      int ldc) {
    double* gp = P.at<double>(L.gpart);
    HIP_TRY((launch_nn<T, T, double, double>(Xa, ld, na, rows, Xb, ld, nb, gp, ldc, (int64_t)ldc * nb, splits, st)));
    HIP_TRY((launch_reduce<double, double>(gp, splits, (int64_t)ldc * nb, ldc, na, nb, C, ldc, st)));
    return RSVD_OK;
  }

  // Sample of the interpolative decompositions (Section 10.4): Y = A X0 (X0: the n x l test matrix), then q times
  // Y = A orth(A^T orth(Y)); leaves Y (m x l panel).
  rsvd_status id_sample_cols(const T* A, int64_t lda, const double* omega_in) {
    const int64_t n = P.d.n;
    const int l = L.l;
    T* omega = P.at<T>(L.omega);
    T* Y = P.at<T>(L.Y);
    T* Q = P.at<T>(L.Q);
    T* Z = P.at<T>(L.Z);
    T* Wp = P.at<T>(L.Wp);
    const int dt = P.d.a_dtype;
    if (omega_in)
      HIP_TRY(launch_rowmajor_to_panel<T>(omega_in, n, l, l, omega, L.ldn, st));
    else
      HIP_TRY(launch_gaussian<T>(P.d.seed, 4u, n, l, 0, omega, 1, L.ldn, st));
    RS_TRY(apply_a(A, lda, omega, l, Y, dt));
    for (int it = 0; it < P.d.q; ++it) {
      RS_TRY(orth(Y, L.ldm, P.d.m, l, L.s_gm, Q));
      RS_TRY(apply_at(A, lda, Q, l, Z, dt));
      RS_TRY(orth(Z, L.ldn, n, l, L.s_gn, Wp));
      RS_TRY(apply_a(A, lda, Wp, l, Y, dt));
    }
    return RSVD_OK;
  }

  // The same for A^T (the row sample of the CUR figure): Z = A^T G (G: m x l, stream 4), then q times
  // Z = A^T orth(A orth(Z)); leaves Z (n x l panel).
  rsvd_status id_sample_rows(const T* A, int64_t lda) {
    const int64_t m = P.d.m;
    const int l = L.l;
    T* Y = P.at<T>(L.Y);
    T* Q = P.at<T>(L.Q);
    T* Z = P.at<T>(L.Z);
    T* Wp = P.at<T>(L.Wp);
    const int dt = P.d.a_dtype;
    HIP_TRY(launch_gaussian<T>(P.d.seed, 4u, m, l, 0, Q, 1, L.ldm, st));
    RS_TRY(apply_at(A, lda, Q, l, Z, dt));
    for (int it = 0; it < P.d.q; ++it) {
      RS_TRY(orth(Z, L.ldn, P.d.n, l, L.s_gn, Wp));
      RS_TRY(apply_a(A, lda, Wp, l, Y, dt));
      RS_TRY(orth(Y, L.ldm, m, l, L.s_gm, Q));
      RS_TRY(apply_at(A, lda, Q, l, Z, dt));
    }
    return RSVD_OK;
  }

  // k steps of column-pivoted QR of the short wide matrix whose columns are the rows of the panel Y (N x nr);
  // pivots into J, S into the plan's S.
  rsvd_status cpqr(const T* Y, int64_t ld, int64_t N, int nr, int k, int* J) {
    HIP_TRY(launch_cpqr<T>(Y, ld, N, nr, k, P.at<double>(L.cp_Q), lp16(nr), P.at<double>(L.cp_S), L.ldS,
                           P.at<double>(L.cp_nrm), P.at<double>(L.cp_orig), P.at<double>(L.cp_bmax),
                           P.at<int>(L.cp_bidx), P.at<unsigned>(L.cp_cnt), J, st));
    return RSVD_OK;
  }

  rsvd_status row_id(const T* A, int64_t lda, const double* omega_in, int32_t* Is, T* X, int64_t ldx) {
    const int k = P.d.k;
    HIP_TRY(launch_fill_int(P.at<int>(L.flags), kFlags, 0, st));
    mark(0);
    RS_TRY(id_sample_cols(A, lda, omega_in));
    mark(1);
    int* J = P.at<int>(L.cp_J);
    RS_TRY(cpqr(P.at<T>(L.Y), L.ldm, P.d.m, L.l, k, J));
    mark(2);
    HIP_TRY(launch_id_solve<T>(P.at<double>(L.cp_S), L.ldS, P.d.m, k, J, P.at<double>(L.cp_small), lp16(k), nullptr,
                               0, X, ldx, st));
    HIP_TRY(hipMemcpyAsync(Is, J, (size_t)k * sizeof(int), hipMemcpyDeviceToDevice, st));
    mark(3);
    mark(4);
    mark(5);
    return RSVD_OK;
  }

  rsvd_status cur(const T* A, int64_t lda, int32_t* Js, double* Uo, int64_t ldu, int32_t* Is) {
    const int64_t m = P.d.m, n = P.d.n;
    const int k = P.d.k, LK = lp16(k);
    int* flags = P.at<int>(L.flags);
    HIP_TRY(launch_fill_int(flags, kFlags, 0, st));
    mark(0);
    RS_TRY(id_sample_rows(A, lda));
    mark(1);
    int* J0 = P.at<int>(L.cp_J);
    int* J1 = J0 + L.LP;
    double* sm = P.at<double>(L.cp_small);
    const size_t K2 = (size_t)L.LP * L.LP;
    double* S11 = sm;
    double* M = sm + K2;
    double* H = sm + 2 * K2;
    double* V = sm + 3 * K2;
    double* T1 = sm + 4 * K2;
    double* lam = sm + 5 * K2;
    double* Zm = P.at<double>(L.cp_Z);
    // [J_s, Z] = column ID of the row sample (its columns are the rows of the n x l panel)
    RS_TRY(cpqr(P.at<T>(L.Z), L.ldn, n, L.l, k, J0));
    HIP_TRY(launch_id_solve<double>(P.at<double>(L.cp_S), L.ldS, n, k, J0, S11, LK, Zm, L.ldn, (double*)nullptr, 0,
                                    st));
    mark(2);
    // I_s = the pivots of A(:, J_s)^T: its columns are the rows of the m x k panel C = A(:, J_s)
    T* C = P.at<T>(L.Q);
    HIP_TRY(launch_gather_cols<T>(A, lda, m, J0, k, C, L.ldm, st));
    RS_TRY(cpqr(C, L.ldm, m, k, k, J1));
    mark(3);
    // U = Z R^+ with R = A(I_s, :): M = Z R^T, H = R R^T = V diag(lam) V^T, U = M V diag(lam)^+ V^T
    double* Rt = P.at<double>(L.Q1d);
    double* gp = P.at<double>(L.gpart);
    HIP_TRY(launch_gather_rows<T>(A, lda, n, J1, k, Rt, L.ldn, st));
    HIP_TRY((launch_nn<double, double, double, double>(Zm, L.ldn, k, n, Rt, L.ldn, k, gp, LK, (int64_t)LK * k, L.s_gn,
                                                       st)));
    HIP_TRY((launch_reduce<double, double>(gp, L.s_gn, (int64_t)LK * k, LK, k, k, M, LK, st)));
    HIP_TRY((launch_nn<double, double, double, double>(Rt, L.ldn, k, n, Rt, L.ldn, k, gp, LK, (int64_t)LK * k, L.s_gn,
                                                       st)));
    HIP_TRY((launch_reduce<double, double>(gp, L.s_gn, (int64_t)LK * k, LK, k, k, H, LK, st)));
    const double tol = small_tol(k);
    // H = R_H^T R_H (Cholesky, R_H into S11, R_H^-1 into T1, both free here); the left singular vectors of
    // R_H^T are H's eigenvectors and sigma^2 its eigenvalues (fewer sweeps than the Jacobi on H's columns)
    HIP_TRY(launch_chol<double>(H, LK, k, LK, tau, T1, S11, nullptr, P.at<double>(L.scr_chol), flags + 8, st));
    HIP_TRY(launch_jacobi<double>(S11, k, LK, tol, 60, lam, V, (double*)nullptr, (double*)nullptr,
                                  P.at<double>(L.scr_jac), flags, st));
    HIP_TRY(launch_square(lam, lam, k, st));
    HIP_TRY(launch_cut_small(lam, k, tol, st));
    HIP_TRY(launch_small_gemm<double>(k, k, k, M, LK, false, V, LK, false, T1, LK, false, lam, st));
    HIP_TRY(launch_small_gemm<double>(k, k, k, T1, LK, false, V, LK, true, H, LK, false, nullptr, st));
    HIP_TRY(launch_transpose64(H, LK, k, k, Uo, ldu, st));
    HIP_TRY(hipMemcpyAsync(Js, J0, (size_t)k * sizeof(int), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(Is, J1, (size_t)k * sizeof(int), hipMemcpyDeviceToDevice, st));
    mark(4);
    mark(5);
    return RSVD_OK;
  }

  // The k dominant left singular vectors of an l-column panel Y (rows x l) in two halves around the Jacobi
  // SVD of R: Y = Q R (CholeskyQR2, Q overwriting Y; R kept in FP64 and transposed into Rc, l x l
  // column-major), W = the left singular vectors of R (Jacobi on its columns), then Q_out = Q W_k and Nt =
  // Y^T Q_out = R^T W_k (l x k, FP64, leading dimension lp16(l)).
  rsvd_status dominant_left_prep(T* Y, int64_t ld, int64_t rows, int l, int splits, double* Rc) {
    const int LPl = lp16(l);
    double* G = P.at<double>(L.G);
    double* R1 = P.at<double>(L.R1);
    double* R = P.at<double>(L.R);
    T* rinv = P.at<T>(L.rinv);
    T* tmp = P.at<T>(L.T);
    int* flags = P.at<int>(L.flags);
    double* scr = P.at<double>(L.scr_chol);
    RS_TRY(gram(Y, ld, rows, l, splits, G));
    HIP_TRY(launch_chol<T>(G, LPl, l, LPl, tau, rinv, R1, nullptr, scr, flags, st));
    HIP_TRY(apply_rinv(Y, ld, rows, l, rinv, LPl, tmp));
    RS_TRY(gram(tmp, ld, rows, l, splits, G));
    HIP_TRY(launch_chol<T>(G, LPl, l, LPl, tau, rinv, R, R1, scr, flags, st));   // R = R2 R1, row-major
    HIP_TRY(apply_rinv(tmp, ld, rows, l, rinv, LPl, Y));
    HIP_TRY(launch_transpose64(R, LPl, l, l, Rc, LPl, st));
    return RSVD_OK;
  }
  rsvd_status dominant_left_finish(const T* Y, int64_t ld, int64_t rows, int l, int k, const double* Rc,
                                   const double* uhat_d, const T* uhat_p, T* Q_out, double* Nt) {
    const int LPl = lp16(l);
    HIP_TRY((launch_tn<T, T, T, T>(Y, ld, l, rows, uhat_p, LPl, k, Q_out, ld, 0, 1, false, st)));
    HIP_TRY(launch_small_gemm<double>(l, k, l, Rc, LPl, true, uhat_d, LPl, false, Nt, LPl, false, nullptr, st));
    return RSVD_OK;
  }

  // Jacobi stopping tolerance for the small FP64 problems of the single pass and the ID/CUR core: n u for FP64
  // data; for FP32 data 1e-10 (the rule of Stage B's small SVD: the data's own rounding is 6e-8).
  double small_tol(int n) const {
    return std::max((double)n * 2.220446049250313e-16, sizeof(T) == 4 ? 1e-10 : 0.0);
  }

  // Single-pass factorisations (Section 5): the general SVD of Section 5.2's figure, or with RSVD_SINGLE_PASS_SYM
  // the symmetric EVD of Section 5.1's figure.  A is read by the sketches only.
  rsvd_status run_single_pass(const T* A, int64_t lda, const double* omega_in, T* U, int64_t ldu, double* S, T* V,
                              int64_t ldv, int kout) {
    const int64_t m = P.d.m, n = P.d.n;
    const int l = L.l, k = P.d.k, LPl = lp16(l), LPk = lp16(k);
    const bool sym = (P.d.flags & RSVD_SINGLE_PASS_SYM) != 0;
    int* flags = P.at<int>(L.flags);
    P.rank_out = kout;
    P.fallback_steps = 0;
    P.err_bound = 0.0;
    P.frob_res = -1.0;
    mark(0);
    HIP_TRY(launch_fill_int(flags, kFlags, 0, st));
    RS_TRY(prep_lowp(A, lda));
    // steps 1-2: test matrices and the sketches Y_c = A G_c, Y_r = A^T G_r
    T* Gc = P.at<T>(L.omega);
    T* Gr = P.at<T>(L.gr);
    T* Yc = P.at<T>(L.Y);
    T* Yr = P.at<T>(L.Z);
    if (omega_in)
      HIP_TRY(launch_rowmajor_to_panel<T>(omega_in, n, l, l, Gc, L.ldn, st));
    else
      HIP_TRY(launch_gaussian<T>(P.d.seed, 4u, n, l, 0, Gc, 1, L.ldn, st));
    if (!sym) HIP_TRY(launch_gaussian<T>(P.d.seed, 11u, m, l, 0, Gr, 1, L.ldm, st));
    if (P.d.sketch_dtype == RSVD_BF16) {
      // the bf16 product rounds its thin operand: round G_c and G_r here, so that the equations of step 4 use
      // the test matrices the sketches were formed with
      if constexpr (sizeof(T) == 4) {
        HIP_TRY(launch_round_bf16(Gc, (int64_t)l * L.ldn, st));
        if (!sym) HIP_TRY(launch_round_bf16(Gr, (int64_t)l * L.ldm, st));
      }
    }
    RS_TRY(apply_a(A, lda, Gc, l, Yc, P.d.sketch_dtype));
    if (!sym) RS_TRY(apply_at(A, lda, Gr, l, Yr, P.d.sketch_dtype));
    mark(1);
    double* sp = P.at<double>(L.sp);
    const size_t L2 = (size_t)L.LP * L.LP;
    double* M1 = sp;
    double* N1 = sp + L2;
    double* M2t = sp + 2 * L2;
    double* N2t = sp + 3 * L2;
    double* P1 = sp + 4 * L2;
    double* P2 = sp + 5 * L2;
    double* Sm = sp + 6 * L2;
    double* Z1 = sp + 7 * L2;
    double* Z2 = sp + 8 * L2;
    double* T1 = sp + 9 * L2;
    double* Cm = sp + 10 * L2;
    double* Wm = sp + 11 * L2;
    double* a1 = sp + 12 * L2;
    double* a2 = a1 + L.LP;
    double* scr = P.at<double>(L.scr_jac);
    const double tol = small_tol(k);
    // step 3: Q_c (Q_r) = the k dominant left singular vectors of Y_c (Y_r); Q_c = (CholeskyQR2 basis of Y_c) x
    // (left singular vectors of its R) stays orthonormal when k exceeds the numerical rank of Y_c, and gives
    // Y_c^T Q_c = R^T W_k without a pass over Y_c.  The two Jacobi SVDs run in one launch.  Equation sets held
    // as l x k panels (FP64): M1 = G_r^T Q_c, N1 = Y_r^T Q_r, M2^T = G_c^T Q_r, N2^T = Y_c^T Q_c (symmetric
    // form: M^T = G^T Q, N^T = Y^T Q in the last two).
    T* Qc = P.at<T>(L.Q);
    T* Qr = P.at<T>(L.Wp);
    double* uhat_d = P.at<double>(L.uhat_d);
    T* uhat_p = P.at<T>(L.uhat_p);
    const double tol_l = small_tol(l);
    RS_TRY(dominant_left_prep(Yc, L.ldm, m, l, L.s_gm, T1));
    if (sym) {
      HIP_TRY(launch_jacobi<T>(T1, l, LPl, tol_l, 60, P.at<double>(L.sigma), uhat_d, uhat_p, (T*)nullptr, scr, flags,
                               st));
      RS_TRY(dominant_left_finish(Yc, L.ldm, m, l, k, T1, uhat_d, uhat_p, Qc, N2t));
    } else {
      // the second problem's outputs in space that step 4 fills later (Cm, Wm, P1, a2)
      RS_TRY(dominant_left_prep(Yr, L.ldn, n, l, L.s_gn, Cm));
      T* uhat_p_r = reinterpret_cast<T*>(P1);
      if (LPl <= 128) {
        const JacobiProblem<T> pc{T1, P.at<double>(L.sigma), uhat_d, uhat_p, nullptr};
        const JacobiProblem<T> pr{Cm, a2, Wm, uhat_p_r, nullptr};
        HIP_TRY(launch_jacobi2<T>(pc, pr, l, LPl, tol_l, 60, flags, st));
      } else {
        HIP_TRY(launch_jacobi<T>(T1, l, LPl, tol_l, 60, P.at<double>(L.sigma), uhat_d, uhat_p, (T*)nullptr, scr,
                                 flags, st));
        HIP_TRY(launch_jacobi<T>(Cm, l, LPl, tol_l, 60, a2, Wm, uhat_p_r, (T*)nullptr, scr, flags, st));
      }
      RS_TRY(dominant_left_finish(Yc, L.ldm, m, l, k, T1, uhat_d, uhat_p, Qc, N2t));
      RS_TRY(dominant_left_finish(Yr, L.ldn, n, l, k, Cm, Wm, uhat_p_r, Qr, N1));
    }
    mark(2);
    // The eigendecompositions of the positive semidefinite P1, P2 go through their Cholesky factors: with
    // P = R^T R, the left singular vectors of R^T are the eigenvectors of P and sigma^2 its eigenvalues (the
    // Jacobi on R^T as in Stage B: fewer sweeps than on the columns of P, and P's condition halved).  R lands
    // in M1 / M2^T (free once P and S are formed), R^-1 in N1; pivots dropped here (k above the rank) count
    // in flags[8..9], not in the sketches' dropped columns.
    double* chol_scr = P.at<double>(L.scr_chol);
    if (sym) {
      RS_TRY(tprod64(Gc, l, Qc, k, L.ldn, n, L.s_gn, M2t, LPl));
      mark(3);
      // P = M M^T, S = N M^T + M N^T
      HIP_TRY(launch_small_gemm<double>(k, k, l, M2t, LPl, true, M2t, LPl, false, P1, LPk, false, nullptr, st));
      HIP_TRY(launch_small_gemm<double>(k, k, l, N2t, LPl, true, M2t, LPl, false, Sm, LPk, false, nullptr, st));
      HIP_TRY(launch_small_gemm<double>(k, k, l, M2t, LPl, true, N2t, LPl, false, Sm, LPk, true, nullptr, st));
      HIP_TRY(launch_chol<double>(P1, LPk, k, LPk, tau, N1, M1, nullptr, chol_scr, flags + 8, st));
      HIP_TRY(launch_jacobi<double>(M1, k, LPk, tol, 60, a1, Z1, (double*)nullptr, (double*)nullptr, scr, flags, st));
      HIP_TRY(launch_square(a1, a1, k, st));
      Z2 = Z1;
      a2 = a1;
    } else {
      RS_TRY(tprod64(Gr, l, Qc, k, L.ldm, m, L.s_gm, M1, LPl));
      RS_TRY(tprod64(Gc, l, Qr, k, L.ldn, n, L.s_gn, M2t, LPl));
      mark(3);
      // P1 = M1^T M1, P2 = M2 M2^T, S = M1^T N1 + N2 M2^T; the two eigendecompositions in one launch
      HIP_TRY(launch_small_gemm<double>(k, k, l, M1, LPl, true, M1, LPl, false, P1, LPk, false, nullptr, st));
      HIP_TRY(launch_small_gemm<double>(k, k, l, M2t, LPl, true, M2t, LPl, false, P2, LPk, false, nullptr, st));
      HIP_TRY(launch_small_gemm<double>(k, k, l, M1, LPl, true, N1, LPl, false, Sm, LPk, false, nullptr, st));
      HIP_TRY(launch_small_gemm<double>(k, k, l, N2t, LPl, true, M2t, LPl, false, Sm, LPk, true, nullptr, st));
      HIP_TRY(launch_chol<double>(P1, LPk, k, LPk, tau, N1, M1, nullptr, chol_scr, flags + 8, st));
      HIP_TRY(launch_chol<double>(P2, LPk, k, LPk, tau, N1, M2t, nullptr, chol_scr, flags + 8, st));
      if (LPk <= 128) {
        const JacobiProblem<double> p1{M1, a1, Z1, nullptr, nullptr};
        const JacobiProblem<double> p2{M2t, a2, Z2, nullptr, nullptr};
        HIP_TRY(launch_jacobi2<double>(p1, p2, k, LPk, tol, 60, flags, st));
      } else {
        HIP_TRY(launch_jacobi<double>(M1, k, LPk, tol, 60, a1, Z1, (double*)nullptr, (double*)nullptr, scr, flags,
                                      st));
        HIP_TRY(launch_jacobi<double>(M2t, k, LPk, tol, 60, a2, Z2, (double*)nullptr, (double*)nullptr, scr, flags,
                                      st));
      }
      HIP_TRY(launch_square(a1, a1, k, st));
      HIP_TRY(launch_square(a2, a2, k, st));
    }
    // P1 C + C P2 = S: C = Z1 [(Z1^T S Z2) ./ (a_i + b_j)] Z2^T
    HIP_TRY(launch_small_gemm<double>(k, k, k, Z1, LPk, true, Sm, LPk, false, T1, LPk, false, nullptr, st));
    HIP_TRY(launch_small_gemm<double>(k, k, k, T1, LPk, false, Z2, LPk, false, Wm, LPk, false, nullptr, st));
    HIP_TRY(launch_sylv_divide(Wm, LPk, k, k, a1, a2, tol, st));
    HIP_TRY(launch_small_gemm<double>(k, k, k, Z1, LPk, false, Wm, LPk, false, T1, LPk, false, nullptr, st));
    HIP_TRY(launch_small_gemm<double>(k, k, k, T1, LPk, false, Z2, LPk, true, Cm, LPk, false, nullptr, st));
    if (sym) HIP_TRY(launch_symmetrize(Cm, LPk, k, st));
    // step 5: C = U_hat D V_hat^T: Jacobi on C gives its left singular vectors and singular values
    double* sigma = P.at<double>(L.sigma);
    T* vhat_p = P.at<T>(L.vhat_p);
    HIP_TRY(launch_jacobi<T>(Cm, k, LPk, tol, 60, sigma, uhat_d, uhat_p, (T*)nullptr, scr, flags, st));
    mark(4);
    // step 6: U = Q_c U_hat; V = Q_r V_hat with V_hat = C^T U_hat diag(sigma)^-1 (symmetric form: V = U and the
    // signed eigenvalues u_hat_j^T C u_hat_j)
    HIP_TRY((launch_tn<T, T, T, T>(Qc, L.ldm, k, m, uhat_p, LPk, kout, U, ldu, 0, 1, true, st)));
    if (sym) {
      HIP_TRY(launch_small_gemm<double>(k, k, k, Cm, LPk, false, uhat_d, LPk, false, Wm, LPk, false, nullptr, st));
      HIP_TRY(launch_coldot(uhat_d, Wm, LPk, k, kout, S, st));
      if (V) HIP_TRY((launch_tn<T, T, T, T>(Qc, L.ldm, k, m, uhat_p, LPk, kout, V, ldv, 0, 1, true, st)));
    } else {
      HIP_TRY(launch_small_gemm<T>(k, k, k, Cm, LPk, true, uhat_d, LPk, false, vhat_p, LPk, false, sigma, st));
      if (V) HIP_TRY((launch_tn<T, T, T, T>(Qr, L.ldn, k, n, vhat_p, LPk, kout, V, ldv, 0, 1, true, st)));
      HIP_TRY(hipMemcpyAsync(S, sigma, (size_t)kout * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    mark(5);
    return RSVD_OK;
  }

  rsvd_status run(const T* A, int64_t lda, const double* omega_in, T* U, int64_t ldu, double* S, T* V, int64_t ldv,
                  int kout) {
    if (P.d.flags & RSVD_NYSTROM) return run_nystrom(A, lda, omega_in, U, ldu, S, V, ldv, kout);
    if (P.d.flags & (RSVD_SINGLE_PASS | RSVD_SINGLE_PASS_SYM))
      return run_single_pass(A, lda, omega_in, U, ldu, S, V, ldv, kout);
    const int64_t m = P.d.m, n = P.d.n;
    const int l = L.l;
    T* omega = P.at<T>(L.omega);
    T* Y = P.at<T>(L.Y);
    T* Q = P.at<T>(L.Q);
    T* Bt = P.at<T>(L.Bt);
    int* flags = P.at<int>(L.flags);
    P.rank_out = kout;
    P.fallback_steps = 0;
    P.err_bound = 0.0;
    P.frob_res = -1.0;
    mark(0);
    HIP_TRY(launch_fill_int(flags, kFlags, 0, st));
    const int sk = P.d.sketch_dtype, pj = P.d.proj_dtype;
    RS_TRY(stage_a(A, lda, omega_in));
    // (7): B = Q^T A, held as B^T (n x l panel).
    RS_TRY(apply_at(A, lda, Q, l, Bt, pj));
    mark(3);
    // (8): SVD of B in FP64.
    RS_TRY(small_svd(l));
    mark(4);
    // (9): U = Q U_hat, V = B^T U_hat D^-1, leading kout columns.
    RS_TRY(lift(l, kout, U, ldu, S, V, ldv));
    mark(5);
    if (P.d.eps <= 0.0) return RSVD_OK;

    // Certificate of Section 14 on the rank-k result, relative to sigma_hat_1.
    const int r = L.r;
    HIP_TRY(launch_gaussian<T>(P.d.seed, 6u, n, r, 0, P.at<T>(L.gc), 1, L.ldn, st));
    {
      const int dt = (sizeof(T) == 8) ? RSVD_F64 : RSVD_F32;
      RS_TRY(apply_a(A, lda, P.at<T>(L.gc), r, P.at<T>(L.agc), dt));
    }
    double sig1 = 0.0;
    HIP_TRY(hipMemcpyAsync(&sig1, P.at<double>(L.sigma), sizeof(double), hipMemcpyDeviceToHost, st));
    double mx = 0.0;
    RS_TRY(cert_residual(A, lda, l, kout, &mx));
    P.err_bound = bound_from(mx);
    const double target = P.d.eps * sig1;
    mark(6);
    if (P.err_bound <= target) { mark(7); return RSVD_OK; }

    // Blocked adaptive range finder (Figure 12) with the residual applied implicitly.
    int lc = l;
    RS_TRY(cert_residual(A, lda, lc, 0, &mx));
    P.err_bound = bound_from(mx);
    const int b = L.b;
    int step = 0;
    T* tmp = P.at<T>(L.tmpr);
    T* C = P.at<T>(L.small);
    while (P.err_bound > target && lc + b <= L.lmax) {
      // b more Gaussian columns: the continuation of Omega's column sequence
      HIP_TRY(launch_gaussian<T>(P.d.seed, 4u, n, b, l + (int64_t)step * b, omega, 1, L.ldn, st));
      RS_TRY(apply_a(A, lda, omega, b, Y, sk));
      for (int pass = 0; pass < 2; ++pass) {   // Y <- (I - Q Q^T) Y, twice
        RS_TRY(panel_tprod(Q, lc, Y, b, L.ldm, m, L.s_gm, C, L.LPmax));
        RS_TRY(panel_mult(Q, lc, L.ldm, m, C, L.LPmax, b, tmp, L.ldm));
        HIP_TRY(launch_axpy_panel<T>(Y, L.ldm, tmp, L.ldm, m, b, T(-1), st));
      }
      T* Qn = Q + (int64_t)lc * L.ldm;
      RS_TRY(orth(Y, L.ldm, m, b, L.s_gm, Qn));
      T* Bn = Bt + (int64_t)lc * L.ldn;
      RS_TRY(apply_at(A, lda, Qn, b, Bn, pj));
      lc += b;
      ++step;
      if (P.d.est_power == 0) {
        // E <- E - Q_new (B_new Gc): the residual sample follows the growth exactly
        RS_TRY(panel_tprod(Bn, b, P.at<T>(L.gc), r, L.ldn, n, L.s_gn, C, L.LPmax));
        RS_TRY(panel_mult(Qn, b, L.ldm, m, C, L.LPmax, r, tmp, L.ldm));
        T* E = P.at<T>(L.E);
        HIP_TRY(launch_axpy_panel<T>(E, L.ldm, tmp, L.ldm, m, r, T(-1), st));
        RS_TRY(max_colnorm(E, &mx));
      } else {
        RS_TRY(cert_residual(A, lda, lc, 0, &mx));
      }
      P.err_bound = bound_from(mx);
    }
    P.fallback_steps = step;
    // Section 12.4: ||A - Q B||_F^2 = ||A||_F^2 - ||B||_F^2 (reported)
    {
      double* fr = P.at<double>(L.frob);
      HIP_TRY(launch_frob2<T>(A, lda, m, n, fr, fr + 1032, st));
      RS_TRY(gram(Bt, L.ldn, n, lc, L.s_gn, P.at<double>(L.G)));
      double a2 = 0.0;
      HIP_TRY(hipMemcpyAsync(&a2, fr + 1032, sizeof(double), hipMemcpyDeviceToHost, st));
      std::vector<double> g((size_t)lp16(lc) * lp16(lc));
      HIP_TRY(hipMemcpyAsync(g.data(), P.at<double>(L.G), g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double b2 = 0.0;
      for (int i = 0; i < lc; ++i) b2 += g[(size_t)i * lp16(lc) + i];
      P.frob_res = sqrt(std::max(a2 - b2, 0.0));
    }
    RS_TRY(small_svd(lc));
    RS_TRY(lift(lc, lc, U, ldu, S, V, ldv));
    P.rank_out = lc;
    mark(7);
    return (P.err_bound <= target) ? RSVD_OK : RSVD_NOT_CERTIFIED;
  }
};

}  // namespace

extern "C" {

const char* rsvd_status_str(int s) {
  switch (s) {
    case RSVD_OK: return "RSVD_OK";
    case RSVD_NOT_CERTIFIED: return "RSVD_NOT_CERTIFIED";
    case RSVD_E_ARG: return "RSVD_E_ARG";
    case RSVD_E_WORKSPACE: return "RSVD_E_WORKSPACE";
    case RSVD_E_HIP: return "RSVD_E_HIP";
    case RSVD_E_NONFINITE: return "RSVD_E_NONFINITE";
    case RSVD_E_UNSUPPORTED: return "RSVD_E_UNSUPPORTED";
    default: return "RSVD_UNKNOWN_STATUS";
  }
}

rsvd_status rsvd_workspace_size(const rsvd_desc* d, size_t* h_bytes) {
  if (!h_bytes || !validate(d)) return RSVD_E_ARG;
  rsvd_status s = supported(d);
  if (s != RSVD_OK) return s;
  *h_bytes = make_layout_any(d).total;
  return RSVD_OK;
}

rsvd_status rsvd_plan(const rsvd_desc* d, void* d_ws, size_t ws_bytes, void* stream, rsvd_plan_t* h_out) {
  if (!h_out || !validate(d)) return RSVD_E_ARG;
  *h_out = nullptr;
  rsvd_status s = supported(d);
  if (s != RSVD_OK) return s;
  Layout L = make_layout_any(d);
  if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return RSVD_E_WORKSPACE;
  rsvd_plan_s* p = new (std::nothrow) rsvd_plan_s();
  if (!p) return RSVD_E_HIP;
  p->d = *d;
  p->L = L;
  p->st = reinterpret_cast<hipStream_t>(stream);
  p->ws = reinterpret_cast<char*>(d_ws);
  p->timing = (d->flags & RSVD_TIMING) != 0;
  if (hipGetDevice(&p->device) != hipSuccess) { delete p; return RSVD_E_HIP; }
  if (p->timing) {
    // Timing-only events (read after the call's stream synchronisation): no system-scope fence, whose cache
    // write-back and invalidation would otherwise stall the next kernel at every event.
    constexpr unsigned kEvFlags = hipEventDisableSystemFence;
    for (int i = 0; i < 8; ++i)
      if (hipEventCreateWithFlags(&p->ev[i], kEvFlags) != hipSuccess) { delete p; return RSVD_E_HIP; }
    for (int i = 0; i < 2 * rsvd_plan_s::kGemmEv; ++i)
      if (hipEventCreateWithFlags(&p->gev[i], kEvFlags) != hipSuccess) { delete p; return RSVD_E_HIP; }
  }
  RSVD_LOGF("plan m=%lld n=%lld l=%d LP=%d splits nn=%d tn=%d gm=%d gn=%d ws=%zu", (long long)d->m,
            (long long)d->n, L.l, L.LP, L.s_nn, L.s_tn, L.s_gm, L.s_gn, L.total);
  *h_out = p;
  return RSVD_OK;
}

void rsvd_destroy(rsvd_plan_t p) {
  if (!p) return;
  if (p->timing) {
    for (int i = 0; i < 8; ++i) (void)hipEventDestroy(p->ev[i]);
    for (int i = 0; i < 2 * rsvd_plan_s::kGemmEv; ++i) (void)hipEventDestroy(p->gev[i]);
  }
  delete p;
}

}  // extern "C"

namespace {

rsvd_status factor_fixed(rsvd_plan_t p, const void* d_A, int64_t lda, const double* d_Omega, void* d_U, int64_t ldu,
                         double* d_S, void* d_V, int64_t ldv, rsvd_info* h_info) {
  const rsvd_desc& d = p->d;
  const int l = d.k + d.p;
  const int kout = (d.flags & RSVD_RETURN_RANK_L) ? l : d.k;
  const int cap = d.eps > 0.0 ? std::max(kout, p->L.lmax) : kout;
  if (lda < d.n || ldu < cap || (d_V && ldv < cap)) return RSVD_E_ARG;
  rsvd_status s;
  p->ngemm = 0;
  if (d.a_dtype == RSVD_F64) {
    Path<double> path(*p);
    s = path.run(static_cast<const double*>(d_A), lda, d_Omega, static_cast<double*>(d_U), ldu, d_S,
                 static_cast<double*>(d_V), ldv, kout);
  } else {
    Path<float> path(*p);
    s = path.run(static_cast<const float*>(d_A), lda, d_Omega, static_cast<float*>(d_U), ldu, d_S,
                 static_cast<float*>(d_V), ldv, kout);
  }
  if (s < 0) return s;
  const bool need_sync = h_info || d.eps > 0.0;
  if (need_sync) {
    int flags[kFlags];
    HIP_TRY(hipMemcpyAsync(flags, p->ws + p->L.flags, sizeof(flags), hipMemcpyDeviceToHost, p->st));
    HIP_TRY(hipStreamSynchronize(p->st));
    if (flags[0] > 0 || flags[4] != 0 || flags[8] > 0) s = RSVD_E_NONFINITE;
    if (h_info) {
      memset(h_info, 0, sizeof(*h_info));
      double s1 = 0.0;
      HIP_TRY(hipMemcpy(&s1, d_S, sizeof(double), hipMemcpyDeviceToHost));
      h_info->p_used = d.p;
      h_info->q_used = d.q;
      h_info->rank_out = p->rank_out;
      h_info->fallback_steps = p->fallback_steps;
      h_info->err_bound = p->err_bound;
      h_info->frob_residual = p->frob_res;
      h_info->sigma1 = s1;
      if (p->timing) {
        for (int i = 0; i < 5; ++i) (void)hipEventElapsedTime(&h_info->stage_ms[i], p->ev[i], p->ev[i + 1]);
        const int last = d.eps > 0.0 ? 7 : 5;
        if (d.eps > 0.0) {
          (void)hipEventElapsedTime(&h_info->stage_ms[5], p->ev[5], p->ev[6]);
          if (p->fallback_steps > 0 || p->rank_out != kout)
            (void)hipEventElapsedTime(&h_info->stage_ms[6], p->ev[6], p->ev[7]);
        }
        (void)hipEventElapsedTime(&h_info->stage_ms[7], p->ev[0], p->ev[last]);
        for (int i = 0; i < p->ngemm; ++i) {
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, p->gev[2 * i], p->gev[2 * i + 1]);
          if (p->gkind[i] == 0) { h_info->nn_ms += ms; h_info->nn_launches++; }
          else { h_info->tn_ms += ms; h_info->tn_launches++; }
        }
      }
      h_info->jacobi_sweeps = flags[3];
      h_info->dropped_cols = (d.flags & RSVD_NYSTROM) ? flags[9] : flags[1];
      h_info->status = s;
    }
    RSVD_LOGF("factor done: status=%d nonfinite=%d dropped=%d jacobi_nonconv=%d bound=%g rank=%d", (int)s, flags[0],
              flags[1], flags[2], p->err_bound, p->rank_out);
  }
  return s;
}

}  // namespace

int rsvd::factor_in_workspace(const void* desc, void* ws, size_t ws_bytes, hipStream_t st, const void* d_A,
                              int64_t lda, const double* d_Omega, void* d_U, int64_t ldu, double* d_S, void* d_V,
                              int64_t ldv) {
  const rsvd_desc* d = static_cast<const rsvd_desc*>(desc);
  if (!validate(d) || !d_A || !d_U || !d_S) return RSVD_E_ARG;
  if (selector_mode(d) || d->eps != 0.0 || (d->flags & RSVD_TIMING)) return RSVD_E_ARG;
  rsvd_status s = supported(d);
  if (s != RSVD_OK) return s;
  rsvd_plan_s p{};
  p.d = *d;
  p.L = make_layout(d);
  if (!ws || p.L.total > ws_bytes || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return RSVD_E_WORKSPACE;
  p.st = st;
  p.ws = static_cast<char*>(ws);
  p.timing = false;
  if (hipGetDevice(&p.device) != hipSuccess) return RSVD_E_HIP;
  return factor_fixed(&p, d_A, lda, d_Omega, d_U, ldu, d_S, d_V, ldv, nullptr);
}

namespace {

// Modelled time (ms) of the plain method at (p, q); see include/rsvd.h.
double sel_cost_ms(int64_t m, int64_t n, int k, int p, int q) {
  const double l = (double)std::min<int64_t>({(int64_t)k + p, m, n});
  const double passes = (2.0 * q + 2.0) * 2.0 * (double)m * (double)n * l * 20.9e-12;
  const double orth = (2.0 * q + 1.0) * 0.104 * pow(std::max(l / 128.0, 1.0), 1.5);
  const double jac = 1.08 * pow(l / 95.0, 1.5);
  return 0.081 + passes + orth + jac;
}

// Grid point of least expected time cost * (2 - prob) among those with prob >= tau (a miss is taken to
// double the time through the fallback); the most probable point if none reaches tau.
void sel_choose(const float* z, int64_t m, int64_t n, int k, float tau, int cap, int* p_out, int* q_out) {
  double best_e = 0.0;
  int best = -1, best_any = -1;
  double best_prob = -1.0;
  for (int iq = 0; iq < kSelNQ; ++iq)
    for (int ip = 0; ip < kSelNP; ++ip) {
      if (k + kSelP[ip] > cap) continue;
      const int o = iq * kSelNP + ip;
      const double prob = 1.0 / (1.0 + exp(-(double)z[o]));
      if (prob > best_prob) { best_prob = prob; best_any = o; }
      if (prob >= tau) {
        const double e = sel_cost_ms(m, n, k, kSelP[ip], iq) * (2.0 - prob);
        if (best < 0 || e < best_e) { best_e = e; best = o; }
      }
    }
  const int o = best >= 0 ? best : best_any;
  *p_out = kSelP[o % kSelNP];
  *q_out = o / kSelNP;
}

// The plan's description and layout swapped for a derived (p, q) during one call.
struct DescSwap {
  rsvd_plan_s* p;
  rsvd_desc d;
  Layout L;
  DescSwap(rsvd_plan_s* pp, const rsvd_desc& e) : p(pp), d(pp->d), L(pp->L) {
    p->d = e;
    p->L = make_layout(&e);
  }
  ~DescSwap() { p->d = d; p->L = L; }
};

rsvd_status probe_run(rsvd_plan_t p, const void* d_A, int64_t lda) {
  if (p->d.a_dtype == RSVD_F64) {
    Path<double> path(*p);
    return path.probe(static_cast<const double*>(d_A), lda);
  }
  Path<float> path(*p);
  return path.probe(static_cast<const float*>(d_A), lda);
}

}  // namespace

extern "C" {

rsvd_status rsvd_factor(rsvd_plan_t p, const void* d_A, int64_t lda, const double* d_Omega, void* d_U, int64_t ldu,
                        double* d_S, void* d_V, int64_t ldv, rsvd_info* h_info) {
  if (!p || !d_A || !d_U || !d_S) return RSVD_E_ARG;
  if (!selector_mode(&p->d)) return factor_fixed(p, d_A, lda, d_Omega, d_U, ldu, d_S, d_V, ldv, h_info);
  // Learned selector: probe, network, decision, then the plain method with the chosen (p, q).
  if (!p->theta || d_Omega || lda < p->d.n) return RSVD_E_ARG;
  rsvd_status s = probe_run(p, d_A, lda);
  if (s != RSVD_OK) return s;
  float* sel = reinterpret_cast<float*>(p->ws + p->L.sel);
  HIP_TRY(launch_mlp_forward(p->theta, 1, sel, sel + 16, sel + 80, sel + 144, p->st));
  float z[40];
  HIP_TRY(hipMemcpyAsync(z, sel + 144, sizeof(z), hipMemcpyDeviceToHost, p->st));
  HIP_TRY(hipStreamSynchronize(p->st));
  int pc = 0, qc = 0;
  sel_choose(z, p->d.m, p->d.n, p->d.k, p->tau, sel_lcap(&p->d), &pc, &qc);
  p->p_used = pc;
  p->q_used = qc;
  DescSwap swap(p, derived_desc(&p->d, pc, qc));
  return factor_fixed(p, d_A, lda, nullptr, d_U, ldu, d_S, d_V, ldv, h_info);
}

// Shared tail of the decomposition entry points: device status words, and h_info when asked for.
static rsvd_status finish_call(rsvd_plan_t p, rsvd_status s, rsvd_info* h_info) {
  if (s < 0 || !h_info) return s;
  int flags[kFlags];
  HIP_TRY(hipMemcpyAsync(flags, p->ws + p->L.flags, sizeof(flags), hipMemcpyDeviceToHost, p->st));
  HIP_TRY(hipStreamSynchronize(p->st));
  if (flags[0] > 0 || flags[4] != 0 || flags[8] > 0) s = RSVD_E_NONFINITE;
  memset(h_info, 0, sizeof(*h_info));
  h_info->p_used = p->d.p;
  h_info->q_used = p->d.q;
  h_info->rank_out = p->d.k;
  h_info->frob_residual = -1.0;
  if (p->timing) {
    for (int i = 0; i < 5; ++i) (void)hipEventElapsedTime(&h_info->stage_ms[i], p->ev[i], p->ev[i + 1]);
    (void)hipEventElapsedTime(&h_info->stage_ms[7], p->ev[0], p->ev[5]);
    for (int i = 0; i < p->ngemm; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, p->gev[2 * i], p->gev[2 * i + 1]);
      if (p->gkind[i] == 0) { h_info->nn_ms += ms; h_info->nn_launches++; }
      else { h_info->tn_ms += ms; h_info->tn_launches++; }
    }
  }
  h_info->jacobi_sweeps = flags[3];
  h_info->dropped_cols = flags[1];
  h_info->status = s;
  return s;
}

rsvd_status rsvd_row_id(rsvd_plan_t p, const void* d_A, int64_t lda, const double* d_Omega, int32_t* d_Is, void* d_X,
                        int64_t ldx, rsvd_info* h_info) {
  if (!p || !d_A || !d_Is || !d_X || !(p->d.flags & RSVD_ID_CUR) || lda < p->d.n || ldx < p->d.k) return RSVD_E_ARG;
  p->ngemm = 0;
  rsvd_status s;
  if (p->d.a_dtype == RSVD_F64) {
    Path<double> path(*p);
    s = path.row_id(static_cast<const double*>(d_A), lda, d_Omega, d_Is, static_cast<double*>(d_X), ldx);
  } else {
    Path<float> path(*p);
    s = path.row_id(static_cast<const float*>(d_A), lda, d_Omega, d_Is, static_cast<float*>(d_X), ldx);
  }
  return finish_call(p, s, h_info);
}

rsvd_status rsvd_cur(rsvd_plan_t p, const void* d_A, int64_t lda, int32_t* d_Js, double* d_U, int64_t ldu,
                     int32_t* d_Is, rsvd_info* h_info) {
  if (!p || !d_A || !d_Js || !d_U || !d_Is || !(p->d.flags & RSVD_ID_CUR) || lda < p->d.n || ldu < p->d.k)
    return RSVD_E_ARG;
  p->ngemm = 0;
  rsvd_status s;
  if (p->d.a_dtype == RSVD_F64) {
    Path<double> path(*p);
    s = path.cur(static_cast<const double*>(d_A), lda, d_Js, d_U, ldu, d_Is);
  } else {
    Path<float> path(*p);
    s = path.cur(static_cast<const float*>(d_A), lda, d_Js, d_U, ldu, d_Is);
  }
  return finish_call(p, s, h_info);
}

rsvd_status rsvd_selector_set(rsvd_plan_t p, const float* d_theta, float tau) {
  if (!p || !d_theta || !(tau > 0.f) || !(tau < 1.f) || !selector_mode(&p->d)) return RSVD_E_ARG;
  p->theta = d_theta;
  p->tau = tau;
  return RSVD_OK;
}

rsvd_status rsvd_probe_sigma(rsvd_plan_t p, const void* d_A, int64_t lda, double* d_sigma16, float* d_x) {
  if (!p || !d_A || !d_sigma16 || lda < p->d.n) return RSVD_E_ARG;
  rsvd_status s = probe_run(p, d_A, lda);
  if (s != RSVD_OK) return s;
  HIP_TRY(hipMemcpyAsync(d_sigma16, p->ws + p->L.sigma, 16 * sizeof(double), hipMemcpyDeviceToDevice, p->st));
  if (d_x) HIP_TRY(hipMemcpyAsync(d_x, p->ws + p->L.sel, 16 * sizeof(float), hipMemcpyDeviceToDevice, p->st));
  return RSVD_OK;
}

rsvd_status rsvd_prefix_bounds(rsvd_plan_t p, const void* d_A, int64_t lda, int32_t n_widths, const int32_t* h_widths,
                               double* h_bounds) {
  if (!p || !d_A || lda < p->d.n || n_widths < 1 || !h_widths || !h_bounds) return RSVD_E_ARG;
  if (selector_mode(&p->d) || !(p->d.eps > 0.0)) return RSVD_E_ARG;
  for (int i = 0; i < n_widths; ++i)
    if (h_widths[i] < 1 || h_widths[i] > p->L.l) return RSVD_E_ARG;
  rsvd_status s;
  p->ngemm = 0;
  if (p->d.a_dtype == RSVD_F64) {
    Path<double> path(*p);
    s = path.prefix_bounds(static_cast<const double*>(d_A), lda, n_widths, h_widths, h_bounds);
  } else {
    Path<float> path(*p);
    s = path.prefix_bounds(static_cast<const float*>(d_A), lda, n_widths, h_widths, h_bounds);
  }
  if (s != RSVD_OK) return s;
  int flags[kFlags];
  HIP_TRY(hipMemcpyAsync(flags, p->ws + p->L.flags, sizeof(flags), hipMemcpyDeviceToHost, p->st));
  HIP_TRY(hipStreamSynchronize(p->st));
  return (flags[0] > 0 || flags[4] != 0) ? RSVD_E_NONFINITE : RSVD_OK;
}

rsvd_status rsvd_mlp_forward(const float* d_theta, int32_t batch, const float* d_X, float* d_H1, float* d_H2,
                             float* d_Z, void* stream) {
  if (!d_theta || batch < 1 || !d_X || !d_H1 || !d_H2 || !d_Z) return RSVD_E_ARG;
  HIP_TRY(launch_mlp_forward(d_theta, batch, d_X, d_H1, d_H2, d_Z, reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_mlp_backward(const float* d_theta, int32_t batch, const float* d_X, const float* d_H1,
                              const float* d_H2, const float* d_Z, const float* d_Y, const float* d_M, float* d_grad,
                              float* d_loss, float* d_scratch, void* stream) {
  if (!d_theta || batch < 1 || !d_X || !d_H1 || !d_H2 || !d_Z || !d_Y || !d_M || !d_grad || !d_loss || !d_scratch)
    return RSVD_E_ARG;
  HIP_TRY(launch_mlp_backward(d_theta, batch, d_X, d_H1, d_H2, d_Z, d_Y, d_M, d_grad, d_loss, d_scratch,
                              reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_mlp_adam(float* d_theta, const float* d_grad, float* d_m, float* d_v, int32_t n, float lr,
                          float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (!d_theta || !d_grad || !d_m || !d_v || n < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return RSVD_E_ARG;
  HIP_TRY(launch_adam(d_theta, d_grad, d_m, d_v, n, lr, beta1, beta2, eps, step, reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_gaussian(uint64_t seed, uint32_t stream_id, int64_t rows, int64_t cols, int64_t col0, int32_t dtype,
                          void* d_out, int64_t ld, void* stream) {
  if (!d_out || rows < 0 || cols < 0 || col0 < 0 || ld < cols) return RSVD_E_ARG;
  if (rows > ((int64_t)1 << 33) || col0 + cols > ((int64_t)1 << 32)) return RSVD_E_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == RSVD_F64)
    HIP_TRY(launch_gaussian<double>(seed, stream_id, rows, cols, col0, static_cast<double*>(d_out), ld, 1, st));
  else if (dtype == RSVD_F32)
    HIP_TRY(launch_gaussian<float>(seed, stream_id, rows, cols, col0, static_cast<float*>(d_out), ld, 1, st));
  else
    return RSVD_E_ARG;
  return RSVD_OK;
}

rsvd_status rsvd_philox4x32_10(int64_t count, const uint32_t* d_ctr, uint32_t k0, uint32_t k1, uint32_t* d_out,
                               void* stream) {
  if (count < 0 || (count > 0 && (!d_ctr || !d_out))) return RSVD_E_ARG;
  HIP_TRY(launch_philox(count, d_ctr, k0, k1, d_out, reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

}  // extern "C"
