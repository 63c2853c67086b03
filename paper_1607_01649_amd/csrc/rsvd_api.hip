// Host runtime behind the C ABI of include/rsvd.h: argument validation,
// workspace carving, split selection and the launch sequence of the
// randomized SVD (Figure 5 of the paper plus Stage B of Section 3).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/rsvd.h"
#include "internal.hpp"

using namespace rsvd;

namespace {

constexpr int kRedGroup = 16;   // partials summed per first-level reduction group
// device status words: [0] non-finite pivot, [1] dropped columns, [2] Jacobi
// not converged, [3] Jacobi sweeps, [4] non-finite entry of A (conversion)
constexpr int kFlags = 64;

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
  int l, LP;
  int64_t ldm, ldn;
  size_t es;   // element size of panels (8 for F64, 4 otherwise)
  int s_nn, s_tn, s_gm, s_gn, s_nn16, s_tn16;
  int64_t ld16, ldT;   // leading dimensions of the bf16 copies of A and A^T
  size_t a16, a16t, omega, Y, T, Q, Z, W, Bt, part, gpart, gpart2, G, R1, R, rinv, rinv_d, Q1d, sigma, uhat_d, uhat_p, vhat_p,
      scr_chol, scr_jac, flags, total;
};

int pick_splits(int64_t tiles, int64_t K, int64_t target, int64_t min_chunk) {
  int64_t s = (target + tiles - 1) / std::max<int64_t>(tiles, 1);
  int64_t cap = std::max<int64_t>(1, K / min_chunk);
  s = std::min(std::max<int64_t>(s, 1), cap);
  return (int)std::min<int64_t>(s, 1024);
}

bool validate(const rsvd_desc* d) {
  if (!d) return false;
  if (d->m < 1 || d->n < 1 || d->k < 1 || d->p < 0 || d->q < 0) return false;
  int64_t l = (int64_t)d->k + d->p;
  if (l > std::min(d->m, d->n) || l > 1024) return false;
  if (d->a_dtype != RSVD_F64 && d->a_dtype != RSVD_F32) return false;
  if (!(d->eps >= 0.0) || !isfinite(d->eps)) return false;
  if (d->n_probe < 0 || d->est_power < 0 || d->fallback_block < 0 || d->max_rank < 0) return false;
  if (d->max_rank > 0 && d->max_rank < l) return false;
  if (d->max_rank > std::min<int64_t>(std::min(d->m, d->n), 1024)) return false;
  if (d->m > (int64_t)1 << 40 || d->n > (int64_t)1 << 40) return false;
  return true;
}

bool uses_bf16(const rsvd_desc* d) { return d->sketch_dtype == RSVD_BF16 || d->proj_dtype == RSVD_BF16; }

rsvd_status supported(const rsvd_desc* d) {
  if (d->a_dtype == RSVD_F64) {
    if (d->sketch_dtype != RSVD_F64 || d->proj_dtype != RSVD_F64) return RSVD_E_UNSUPPORTED;
  } else {
    auto ok = [](int t) { return t == RSVD_F32 || t == RSVD_BF16; };
    if (!ok(d->sketch_dtype) || !ok(d->proj_dtype)) return RSVD_E_UNSUPPORTED;
  }
  if (d->eps > 0.0) return RSVD_E_UNSUPPORTED;
  return RSVD_OK;
}

Layout make_layout(const rsvd_desc* d) {
  Layout L{};
  L.l = d->k + d->p;
  L.LP = (int)round_up(L.l, 16);
  L.ldm = round_up(d->m, 64);
  L.ldn = round_up(d->n, 64);
  L.es = (d->a_dtype == RSVD_F64) ? 8 : 4;
  const int64_t cg = (L.l + 127) / 128;
  L.s_nn = pick_splits(((d->m + 127) / 128) * cg, d->n, 2048, 512);
  L.s_tn = pick_splits(((d->n + 255) / 256) * cg, d->m, 2048, 512);
  const int64_t gt = ((L.l + 127) / 128) * cg;
  L.s_gm = pick_splits(gt, d->m, 512, 128);
  L.s_gn = pick_splits(gt, d->n, 512, 128);
  L.s_nn = nn_splits_used(d->n, L.s_nn);
  L.s_tn = nn_splits_used(d->m, L.s_tn);
  L.s_gm = nn_splits_used(d->m, L.s_gm);
  L.s_gn = nn_splits_used(d->n, L.s_gn);
  L.s_nn16 = lp_splits_used(d->n, L.s_nn);
  L.s_tn16 = lp_splits_used(d->m, L.s_tn);
  L.ld16 = round_up(d->n, 128);
  L.ldT = round_up(d->m, 128);
  const size_t LP = (size_t)L.LP;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = round_up(off + bytes, 256); return o; };
  const bool b16 = uses_bf16(d);
  L.a16 = take(b16 ? (size_t)d->m * L.ld16 * 2 : 256);
  L.a16t = take(b16 ? (size_t)d->n * L.ldT * 2 : 256);
  L.omega = take(LP * L.ldn * L.es);
  L.Y = take(LP * L.ldm * L.es);
  L.T = take(LP * std::max(L.ldm, L.ldn) * L.es);
  L.Q = take(LP * L.ldm * L.es);
  L.Z = take(LP * L.ldn * L.es);
  L.W = take(LP * L.ldn * L.es);
  L.Bt = take(LP * L.ldn * L.es);
  L.part = take(std::max(std::max((size_t)L.s_nn, (size_t)L.s_nn16) * LP * L.ldm,
                          std::max((size_t)L.s_tn, (size_t)L.s_tn16) * LP * L.ldn) * L.es);
  L.gpart = take((size_t)std::max(L.s_gm, L.s_gn) * LP * LP * 8);
  L.gpart2 = take((size_t)((std::max(L.s_gm, L.s_gn) + kRedGroup - 1) / kRedGroup) * LP * LP * 8);
  L.G = take(LP * LP * 8);
  L.R1 = take(LP * LP * 8);
  L.R = take(LP * LP * 8);
  L.rinv = take(LP * LP * L.es);
  L.rinv_d = take(LP * LP * 8);
  L.Q1d = take(LP * L.ldn * 8);
  L.sigma = take(LP * 8);
  L.uhat_d = take(LP * LP * 8);
  L.uhat_p = take(LP * LP * L.es);
  L.vhat_p = take(LP * LP * L.es);
  L.scr_chol = take(LP > 128 ? LP * LP * 8 : 256);
  L.scr_jac = take(LP > 128 ? LP * LP * 8 : 256);
  L.flags = take(kFlags * sizeof(int));
  L.total = off;
  return L;
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
  static constexpr int kGemmEv = 64;          // event pairs around A-products (RSVD_TIMING)
  hipEvent_t gev[2 * kGemmEv];
  int gkind[kGemmEv];                         // 0 = A*X, 1 = A^T*X
  mutable int ngemm = 0;
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

template <typename T> struct Path {
  const rsvd_plan_s& P;
  const Layout& L;
  hipStream_t st;
  int l, LP;
  double tau;
  explicit Path(const rsvd_plan_s& p) : P(p), L(p.L), st(p.st), l(p.L.l), LP(p.L.LP) {
    const double u = sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
    tau = (double)l * u * u;
  }

  // G = X^T X for an l-column panel X with `rows` rows (FP64 accumulation).
  rsvd_status gram(const T* X, int64_t ldx, int64_t rows, int splits, double* G) {
    double* gp = P.at<double>(L.gpart);
    HIP_TRY((launch_nn<T, T, double, double>(X, ldx, l, rows, X, ldx, l, gp, LP, (int64_t)LP * LP, splits, st)));
    HIP_TRY(launch_reduce2<double>(gp, splits, kRedGroup, (int64_t)LP * LP, LP, l, l, P.at<double>(L.gpart2), G, LP,
                                   st));
    return RSVD_OK;
  }

  // out = orth(X): CholeskyQR2 (two passes of G = X^T X = R^T R, X <- X R^-1).
  rsvd_status orth(const T* X, int64_t ld, int64_t rows, int splits, T* out) {
    double* G = P.at<double>(L.G);
    T* rinv = P.at<T>(L.rinv);
    T* tmp = P.at<T>(L.T);
    int* flags = P.at<int>(L.flags);
    double* scr = P.at<double>(L.scr_chol);
    rsvd_status s;
    if ((s = gram(X, ld, rows, splits, G)) != RSVD_OK) return s;
    HIP_TRY(launch_chol<T>(G, LP, l, LP, tau, rinv, nullptr, nullptr, scr, flags, st));
    HIP_TRY((launch_tn<T, T, T, T>(X, ld, l, rows, rinv, LP, l, tmp, ld, 0, 1, false, st)));
    if ((s = gram(tmp, ld, rows, splits, G)) != RSVD_OK) return s;
    HIP_TRY(launch_chol<T>(G, LP, l, LP, tau, rinv, nullptr, nullptr, scr, flags, st));
    HIP_TRY((launch_tn<T, T, T, T>(tmp, ld, l, rows, rinv, LP, l, out, ld, 0, 1, false, st)));
    return RSVD_OK;
  }

  // Y = A X (m x l panel) for an n-row panel X, operands in precision `dt`.
  rsvd_status apply_a(const T* A, int64_t lda, const T* X, T* Y, int dt) {
    T* part = P.at<T>(L.part);
    const int64_t m = P.d.m, n = P.d.n;
    int S = L.s_nn;
    int ev = gemm_begin(0);
    if (dt == RSVD_BF16) {
      if constexpr (sizeof(T) == 4) {
        S = L.s_nn16;
        HIP_TRY(launch_nn_bf16(P.at<uint16_t>(L.a16), L.ld16, m, n, X, L.ldn, l, part, L.ldm, (int64_t)LP * L.ldm, S,
                               st));
      }
    } else {
      HIP_TRY((launch_nn<T, T, T, T>(A, lda, m, n, X, L.ldn, l, part, L.ldm, (int64_t)LP * L.ldm, S, st)));
    }
    gemm_end(ev);
    HIP_TRY((launch_reduce<T, T>(part, S, (int64_t)LP * L.ldm, L.ldm, m, l, Y, L.ldm, st)));
    return RSVD_OK;
  }

  // Z = A^T Q (n x l panel) for an m-row panel Q, operands in precision `dt`.
  rsvd_status apply_at(const T* A, int64_t lda, const T* Qp, T* Z, int dt) {
    T* part = P.at<T>(L.part);
    const int64_t m = P.d.m, n = P.d.n;
    int S = L.s_tn;
    int ev = gemm_begin(1);
    if (dt == RSVD_BF16) {
      if constexpr (sizeof(T) == 4) {
        S = L.s_tn16;
        HIP_TRY(launch_nn_bf16(P.at<uint16_t>(L.a16t), L.ldT, n, m, Qp, L.ldm, l, part, L.ldn, (int64_t)LP * L.ldn, S,
                               st));
      }
    } else {
      HIP_TRY((launch_tn<T, T, T, T>(A, lda, m, n, Qp, L.ldm, l, part, L.ldn, (int64_t)LP * L.ldn, S, false, st)));
    }
    gemm_end(ev);
    HIP_TRY((launch_reduce<T, T>(part, S, (int64_t)LP * L.ldn, L.ldn, n, l, Z, L.ldn, st)));
    return RSVD_OK;
  }

  void mark(int i) { if (P.timing) (void)hipEventRecord(P.ev[i], st); }
  int gemm_begin(int kind) {
    if (!P.timing || P.ngemm >= rsvd_plan_s::kGemmEv) return -1;
    int i = P.ngemm++;
    const_cast<rsvd_plan_s&>(P).gkind[i] = kind;
    (void)hipEventRecord(P.gev[2 * i], st);
    return i;
  }
  void gemm_end(int i) { if (i >= 0) (void)hipEventRecord(P.gev[2 * i + 1], st); }

  rsvd_status run(const T* A, int64_t lda, const double* omega_in, T* U, int64_t ldu, double* S, T* V, int64_t ldv,
                  int kout) {
    const int64_t m = P.d.m, n = P.d.n;
    T* omega = P.at<T>(L.omega);
    T* Y = P.at<T>(L.Y);
    T* Q = P.at<T>(L.Q);
    T* Z = P.at<T>(L.Z);
    T* W = P.at<T>(L.W);
    T* Bt = P.at<T>(L.Bt);
    int* flags = P.at<int>(L.flags);
    rsvd_status s;
    mark(0);
    HIP_TRY(launch_fill_int(flags, kFlags, 0, st));
    const int sk = P.d.sketch_dtype, pj = P.d.proj_dtype;
    if (uses_bf16(&P.d)) {
      if constexpr (sizeof(T) == 4)
        HIP_TRY(launch_to_bf16(A, lda, m, n, P.at<uint16_t>(L.a16), L.ld16, P.at<uint16_t>(L.a16t), L.ldT, flags + 4,
                               st));
    }
    // Figure 5 (1): Gaussian test matrix.
    if (omega_in)
      HIP_TRY(launch_rowmajor_to_panel<T>(omega_in, n, l, l, omega, L.ldn, st));
    else
      HIP_TRY(launch_gaussian<T>(P.d.seed, 4u, n, l, 0, omega, 1, L.ldn, st));
    // (2): Q = orth(A Omega).
    if ((s = apply_a(A, lda, omega, Y, sk)) != RSVD_OK) return s;
    if ((s = orth(Y, L.ldm, m, L.s_gm, Q)) != RSVD_OK) return s;
    mark(1);
    // (3)-(6): q power steps with re-orthonormalisation.
    for (int it = 0; it < P.d.q; ++it) {
      if ((s = apply_at(A, lda, Q, Z, sk)) != RSVD_OK) return s;
      if ((s = orth(Z, L.ldn, n, L.s_gn, W)) != RSVD_OK) return s;
      if ((s = apply_a(A, lda, W, Y, sk)) != RSVD_OK) return s;
      if ((s = orth(Y, L.ldm, m, L.s_gm, Q)) != RSVD_OK) return s;
    }
    mark(2);
    // (7): B = Q^T A, held as B^T (n x l panel).
    if ((s = apply_at(A, lda, Q, Bt, pj)) != RSVD_OK) return s;
    mark(3);
    // (8): SVD of B in FP64: B^T = Q_B R by CholeskyQR2, then Jacobi on R^T.
    {
      double* G = P.at<double>(L.G);
      double* R1 = P.at<double>(L.R1);
      double* R = P.at<double>(L.R);
      double* rinv_d = P.at<double>(L.rinv_d);
      double* Q1d = P.at<double>(L.Q1d);
      double* gp = P.at<double>(L.gpart);
      double* scr = P.at<double>(L.scr_chol);
      double* gp2 = P.at<double>(L.gpart2);
      HIP_TRY((launch_nn<T, T, double, double>(Bt, L.ldn, l, n, Bt, L.ldn, l, gp, LP, (int64_t)LP * LP, L.s_gn, st)));
      HIP_TRY(launch_reduce2<double>(gp, L.s_gn, kRedGroup, (int64_t)LP * LP, LP, l, l, gp2, G, LP, st));
      HIP_TRY(launch_chol<double>(G, LP, l, LP, tau, rinv_d, R1, nullptr, scr, flags, st));
      HIP_TRY((launch_tn<T, double, double, double>(Bt, L.ldn, l, n, rinv_d, LP, l, Q1d, L.ldn, 0, 1, false, st)));
      HIP_TRY((launch_nn<double, double, double, double>(Q1d, L.ldn, l, n, Q1d, L.ldn, l, gp, LP, (int64_t)LP * LP,
                                                         L.s_gn, st)));
      HIP_TRY(launch_reduce2<double>(gp, L.s_gn, kRedGroup, (int64_t)LP * LP, LP, l, l, gp2, G, LP, st));
      HIP_TRY(launch_chol<double>(G, LP, l, LP, tau, rinv_d, R, R1, scr, flags, st));
      const double tol = (double)l * 2.220446049250313e-16;
      HIP_TRY(launch_jacobi<T>(R, l, LP, tol, 60, P.at<double>(L.sigma), P.at<double>(L.uhat_d), P.at<T>(L.uhat_p),
                               P.at<T>(L.vhat_p), P.at<double>(L.scr_jac), flags, st));
    }
    mark(4);
    // (9): U = Q U_hat and V = B^T U_hat D^-1, leading kout columns, row-major.
    HIP_TRY((launch_tn<T, T, T, T>(Q, L.ldm, l, m, P.at<T>(L.uhat_p), LP, kout, U, ldu, 0, 1, true, st)));
    if (V) HIP_TRY((launch_tn<T, T, T, T>(Bt, L.ldn, l, n, P.at<T>(L.vhat_p), LP, kout, V, ldv, 0, 1, true, st)));
    HIP_TRY(hipMemcpyAsync(S, P.at<double>(L.sigma), (size_t)kout * sizeof(double), hipMemcpyDeviceToDevice, st));
    mark(5);
    return RSVD_OK;
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
    case RSVD_E_BREAKDOWN: return "RSVD_E_BREAKDOWN";
    default: return "RSVD_UNKNOWN_STATUS";
  }
}

rsvd_status rsvd_workspace_size(const rsvd_desc* d, size_t* h_bytes) {
  if (!h_bytes || !validate(d)) return RSVD_E_ARG;
  rsvd_status s = supported(d);
  if (s != RSVD_OK) return s;
  *h_bytes = make_layout(d).total;
  return RSVD_OK;
}

rsvd_status rsvd_plan(const rsvd_desc* d, void* d_ws, size_t ws_bytes, void* stream, rsvd_plan_t* h_out) {
  if (!h_out || !validate(d)) return RSVD_E_ARG;
  *h_out = nullptr;
  rsvd_status s = supported(d);
  if (s != RSVD_OK) return s;
  Layout L = make_layout(d);
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
    for (int i = 0; i < 8; ++i)
      if (hipEventCreate(&p->ev[i]) != hipSuccess) { delete p; return RSVD_E_HIP; }
    for (int i = 0; i < 2 * rsvd_plan_s::kGemmEv; ++i)
      if (hipEventCreate(&p->gev[i]) != hipSuccess) { delete p; return RSVD_E_HIP; }
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

rsvd_status rsvd_factor(rsvd_plan_t p, const void* d_A, int64_t lda, const double* d_Omega, void* d_U, int64_t ldu,
                        double* d_S, void* d_V, int64_t ldv, rsvd_info* h_info) {
  if (!p || !d_A || !d_U || !d_S) return RSVD_E_ARG;
  const rsvd_desc& d = p->d;
  const int l = d.k + d.p;
  const int kout = (d.flags & RSVD_RETURN_RANK_L) ? l : d.k;
  if (lda < d.n || ldu < kout || (d_V && ldv < kout)) return RSVD_E_ARG;
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
  if (s != RSVD_OK) return s;
  if (h_info) {
    memset(h_info, 0, sizeof(*h_info));
    int flags[kFlags];
    HIP_TRY(hipMemcpyAsync(flags, p->ws + p->L.flags, sizeof(flags), hipMemcpyDeviceToHost, p->st));
    HIP_TRY(hipStreamSynchronize(p->st));
    double s1 = 0.0;
    HIP_TRY(hipMemcpy(&s1, d_S, sizeof(double), hipMemcpyDeviceToHost));
    h_info->p_used = d.p;
    h_info->q_used = d.q;
    h_info->rank_out = kout;
    h_info->sigma1 = s1;
    h_info->orth_retries = 0;
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
    if (flags[0] > 0 || flags[4] != 0) s = RSVD_E_NONFINITE;
    h_info->status = s;
    RSVD_LOGF("factor done: nonfinite=%d dropped=%d jacobi_nonconv=%d", flags[0], flags[1], flags[2]);
  }
  return s;
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
