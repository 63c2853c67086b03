// Kernel-level C entry points (include/rsvd_kernels.h): each building block of
// the randomized SVD callable on its own, for per-kernel parity tests.
#include "../../include/rsvd_kernels.h"
#include "internal.hpp"

#include <algorithm>

using namespace rsvd;

#define K_TRY(expr)                           \
  do {                                        \
    if ((expr) != hipSuccess) return RSVD_E_HIP; \
  } while (0)

extern "C" {

rsvd_status rsvd_k_product_nn(int32_t prec, int64_t rows, int64_t K, const void* A, int64_t lda, const void* X,
                              int64_t ldx, int32_t ncols, void* out, int64_t ldo, void* stream) {
  if (!A || !X || !out || rows < 1 || K < 1 || ncols < 1 || ncols > 1024 || lda < K || ldx < K || ldo < rows)
    return RSVD_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (prec == RSVD_F64)
    K_TRY((launch_nn<double, double, double, double>((const double*)A, lda, rows, K, (const double*)X, ldx, ncols,
                                                     (double*)out, ldo, 0, 1, s)));
  else if (prec == RSVD_F32)
    K_TRY((launch_nn<float, float, float, float>((const float*)A, lda, rows, K, (const float*)X, ldx, ncols,
                                                 (float*)out, ldo, 0, 1, s)));
  else if (prec == RSVD_F32_ACC64)
    K_TRY((launch_nn<float, float, double, double>((const float*)A, lda, rows, K, (const float*)X, ldx, ncols,
                                                   (double*)out, ldo, 0, 1, s)));
  else
    return RSVD_E_ARG;
  return RSVD_OK;
}

rsvd_status rsvd_k_gram(int32_t prec, int64_t K, int32_t nc, const void* Y, int64_t ldy, double* G, int64_t ldg,
                        void* stream) {
  if (!Y || !G || K < 1 || nc < 1 || nc > 1024 || ldy < K || (ldy % 64) != 0 || ldg < nc) return RSVD_E_ARG;
  if ((reinterpret_cast<uintptr_t>(Y) & 15) != 0) return RSVD_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (prec == RSVD_F32)
    K_TRY(launch_gram<float>((const float*)Y, ldy, K, nc, G, ldg, 0, 1, s));
  else if (prec == RSVD_F64)
    K_TRY(launch_gram<double>((const double*)Y, ldy, K, nc, G, ldg, 0, 1, s));
  else
    return RSVD_E_ARG;
  return RSVD_OK;
}

rsvd_status rsvd_k_product_tn(int32_t prec, int64_t K, int64_t N, const void* A, int64_t lda, const void* P,
                              int64_t ldp, int32_t ncols, void* out, int64_t ldo, int32_t out_rowmajor,
                              void* stream) {
  if (!A || !P || !out || K < 1 || N < 1 || ncols < 1 || ncols > 1024 || lda < N || ldp < K) return RSVD_E_ARG;
  if (out_rowmajor ? (ldo < ncols) : (ldo < N)) return RSVD_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bool rm = out_rowmajor != 0;
  if (prec == RSVD_F64)
    K_TRY((launch_tn<double, double, double, double>((const double*)A, lda, K, N, (const double*)P, ldp, ncols,
                                                     (double*)out, ldo, 0, 1, rm, s)));
  else if (prec == RSVD_F32)
    K_TRY((launch_tn<float, float, float, float>((const float*)A, lda, K, N, (const float*)P, ldp, ncols,
                                                 (float*)out, ldo, 0, 1, rm, s)));
  else
    return RSVD_E_ARG;
  return RSVD_OK;
}

rsvd_status rsvd_k_scratch_bytes(int32_t l, size_t* h_bytes) {
  if (!h_bytes || l < 1 || l > 1024) return RSVD_E_ARG;
  const int LP = (l + 15) / 16 * 16;
  *h_bytes = LP <= 128 ? 0 : std::max(chol_blocked_scratch_doubles(LP) * sizeof(double),
                                      jacobi_blocked_scratch_bytes(LP));
  return RSVD_OK;
}

rsvd_status rsvd_k_cholesky(int32_t l, const double* G, int64_t ldg, double tau_rel, double* Rinv, double* R,
                            int32_t* flags, void* scratch, void* stream) {
  if (l < 1 || l > 1024 || !G || !Rinv || !R || !flags || ldg < l || !(tau_rel >= 0.0)) return RSVD_E_ARG;
  int LP = (l + 15) / 16 * 16;
  if (LP > 128 && !scratch) return RSVD_E_ARG;
  K_TRY(launch_chol<double>(G, ldg, l, LP, tau_rel, Rinv, R, nullptr, reinterpret_cast<double*>(scratch), flags,
                            reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_k_small_svd(int32_t l, const double* R, double* sigma, double* Uhat, int32_t* flags,
                             void* scratch, void* stream) {
  if (l < 1 || l > 1024 || !R || !sigma || !Uhat || !flags) return RSVD_E_ARG;
  int LP = (l + 15) / 16 * 16;
  if (LP > 128 && !scratch) return RSVD_E_ARG;
  K_TRY(launch_jacobi<double>(R, l, LP, (double)l * 2.220446049250313e-16, 60, sigma, Uhat, (double*)nullptr,
                              (double*)nullptr, reinterpret_cast<double*>(scratch), flags,
                              reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_k_convert_bf16(int64_t m, int64_t n, const float* A, int64_t lda, uint16_t* A16, int64_t ld16,
                                uint16_t* A16T, int64_t ldT, int32_t* flag, void* stream) {
  if (!A || !A16 || !A16T || !flag || m < 1 || n < 1 || lda < n || ld16 < n || ldT < m || ld16 % 128 || ldT % 128)
    return RSVD_E_ARG;
  K_TRY(launch_to_bf16(A, lda, m, n, A16, ld16, A16T, ldT, flag, reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_k_lp_scratch_bytes(int32_t dtype, int64_t K, int32_t ncols, size_t* h_bytes) {
  if (!h_bytes || K < 1 || ncols < 1 || ncols > 1024 || (dtype != RSVD_BF16 && dtype != RSVD_FP8_E4M3))
    return RSVD_E_ARG;
  *h_bytes = lp_scratch_bytes(dtype == RSVD_BF16 ? 0 : 1, K, ncols);
  return RSVD_OK;
}

rsvd_status rsvd_k_product_bf16(int64_t rows, int64_t K, const uint16_t* A16, int64_t lda, const float* X, int64_t ldx,
                                int32_t ncols, float* out, int64_t ldo, void* scratch, void* stream) {
  if (!A16 || !X || !out || !scratch || rows < 1 || K < 1 || ncols < 1 || ncols > 1024 || lda < K || lda % 128 ||
      ldx < K || ldo < rows || (reinterpret_cast<uintptr_t>(scratch) & 255))
    return RSVD_E_ARG;
  K_TRY(launch_nn_lp(0, false, A16, lda, nullptr, 0, 0, rows, K, X, ldx, ncols, scratch, out, ldo, 0, 1,
                     reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_k_convert_fp8(int64_t m, int64_t n, const float* A, int64_t lda, uint8_t* A8, int64_t ld8,
                               uint8_t* A8T, int64_t ldT, float* scale, int32_t* flag, void* stream) {
  if (!A || !A8 || !A8T || !scale || !flag || m < 1 || n < 1 || lda < n || ld8 < n || ldT < m || ld8 % 128 ||
      ldT % 128)
    return RSVD_E_ARG;
  K_TRY(launch_to_fp8(A, lda, m, n, A8, ld8, A8T, ldT, scale, flag, reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_k_product_fp8(int64_t rows, int64_t K, const uint8_t* A8, int64_t lda, const float* scale,
                               int64_t s_row, int64_t s_k, const float* X, int64_t ldx, int32_t ncols, float* out,
                               int64_t ldo, void* scratch, void* stream) {
  if (!A8 || !scale || !X || !out || !scratch || rows < 1 || K < 1 || ncols < 1 || ncols > 1024 || lda < K ||
      lda % 128 || ldx < K || ldo < rows || s_row < 0 || s_k < 0 || (reinterpret_cast<uintptr_t>(scratch) & 255))
    return RSVD_E_ARG;
  K_TRY(launch_nn_lp(1, false, A8, lda, scale, s_row, s_k, rows, K, X, ldx, ncols, scratch, out, ldo, 0, 1,
                     reinterpret_cast<hipStream_t>(stream)));
  return RSVD_OK;
}

rsvd_status rsvd_k_srht_sketch(int32_t prec, int64_t m, int64_t n, const void* A, int64_t lda, int32_t l,
                               uint64_t seed, void* signs, int32_t* subset, void* Y, int64_t ldy, void* stream) {
  if (!A || !signs || !subset || !Y || m < 1 || n < 1 || lda < n || l < 1 || l > 1024 || ldy < l) return RSVD_E_ARG;
  if (prec != RSVD_F32 && prec != RSVD_F64) return RSVD_E_ARG;
  if (n > srht_max_n(prec == RSVD_F64 ? 8 : 4)) return RSVD_E_ARG;
  int64_t N = 1;
  while (N < n) N *= 2;
  if (l > N) return RSVD_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (prec == RSVD_F64) {
    K_TRY(launch_srht_setup<double>(seed, (int)n, l, (double*)signs, subset, s));
    K_TRY(launch_srht_sketch<double>((const double*)A, lda, m, (int)n, (const double*)signs, subset, l, (double*)Y,
                                     ldy, 1, s));
  } else {
    K_TRY(launch_srht_setup<float>(seed, (int)n, l, (float*)signs, subset, s));
    K_TRY(launch_srht_sketch<float>((const float*)A, lda, m, (int)n, (const float*)signs, subset, l, (float*)Y, ldy,
                                    1, s));
  }
  return RSVD_OK;
}

}  // extern "C"
