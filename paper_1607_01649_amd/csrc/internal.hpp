// Internal launch wrappers of the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace rsvd {

// rng.hip
hipError_t launch_philox(int64_t count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t s);
template <typename T>
hipError_t launch_gaussian(uint64_t seed, uint32_t stream, int64_t rows, int64_t cols, int64_t col0, T* out,
                           int64_t row_stride, int64_t col_stride, hipStream_t s);

// gemm.hip -- see the file comment for the panel layout.
// nn: out[s][c][r] = sum_{j in split s} A[r][j] X(j, c); A rows x K row-major, X panel (X[c*ldx + j]).
template <typename TA, typename TX, typename TC, typename TO>
hipError_t launch_nn(const TA* A, int64_t lda, int64_t rows, int64_t K, const TX* X, int64_t ldx, int ncols, TO* out,
                     int64_t ldo, int64_t part_stride, int splits, hipStream_t s);
// out = A P with P upper triangular (P(i, c) = 0 for i > c); layouts as launch_tn with one range.  skip
// (optional): when *skip is set on the device the product goes to out_skip instead of out, or nowhere when
// out_skip is null (the two applies of a CholeskyQR whose second pass is skipped: the first writes the final
// basis, the second nothing).
hipError_t launch_apply_upper(const float* A, int64_t lda, int64_t K, int64_t N, const float* P, int64_t ldp,
                              int ncols, float* out, int64_t ldo, hipStream_t s, const int* skip = nullptr,
                              float* out_skip = nullptr);
hipError_t launch_apply_upper(const float* A, int64_t lda, int64_t K, int64_t N, const double* P, int64_t ldp,
                              int ncols, double* out, int64_t ldo, hipStream_t s);
hipError_t launch_apply_upper(const double* A, int64_t lda, int64_t K, int64_t N, const double* P, int64_t ldp,
                              int ncols, double* out, int64_t ldo, hipStream_t s, const int* skip = nullptr,
                              double* out_skip = nullptr);
// tn: out[s][c][j] = sum_{i in split s} A[i][j] P(i, c); A K x N row-major, P panel (P[c*ldp + i]).
template <typename TA, typename TP, typename TC, typename TO>
hipError_t launch_tn(const TA* A, int64_t lda, int64_t K, int64_t N, const TP* P, int64_t ldp, int ncols, TO* out,
                     int64_t ldo, int64_t part_stride, int splits, bool out_rowmajor, hipStream_t s);
int nn_splits_used(int64_t K, int splits);
template <typename TP, typename TO>
hipError_t launch_reduce(const TP* part, int S, int64_t pstride, int64_t ldp, int64_t rows, int ncols, TO* out,
                         int64_t ldo, hipStream_t s, const int* skip = nullptr);
template <typename TP>
hipError_t launch_reduce2(const TP* part, int S, int group, int64_t pstride, int64_t ldp, int64_t rows, int ncols,
                          TP* tmp, TP* out, int64_t ldo, hipStream_t s, const int* skip = nullptr);

// chol.hip.  skip_out (optional): 1 when the factor shows the panel well enough conditioned that one
// CholeskyQR pass suffices (scaled Frobenius condition bound at most kappa_max); skip_in (optional): when
// *skip_in is set the call only writes R^-1 = I (a skipped second pass; r_out must be null).
template <typename TQ>
hipError_t launch_chol(const double* g, int64_t ldg, int l, int LP, double tau_rel, TQ* rinv_p, double* r_out,
                       const double* r_prev, double* scratch, int* flags, hipStream_t s, int* skip_out = nullptr,
                       double kappa_max = 0.0, const int* skip_in = nullptr);

// blocked.hip -- the same factorisations for l > 128, spread over many workgroups.
size_t chol_blocked_scratch_doubles(int LP);
template <typename TQ>
hipError_t launch_chol_blocked(const double* g, int64_t ldg, int l, int LP, double tau, TQ* rinv_p, double* r_out,
                               const double* r_prev, double* scratch, int* flags, hipStream_t s,
                               int* skip_out = nullptr, double kappa2_max = 0.0, const int* skip_in = nullptr);
// 64 x 64 diagonal block of the blocked Cholesky (chol.hip): R_JJ into M, S_JJ = R_JJ^-1 into X.
hipError_t launch_chol_diag64(double* M, int LB, int j0, int l, const double* gdiag, double tau_rel, double* X,
                              int* flags, hipStream_t s, const int* skip = nullptr);
size_t jacobi_blocked_scratch_bytes(int LP);
template <typename TU>
hipError_t launch_jacobi_blocked(const double* R, int l, int LP, double tol, int max_sweeps, double* sigma,
                                 double* uhat_d, TU* uhat_p, TU* vhat_p, double* scratch, int* flags, hipStream_t s);
template <typename TU>
hipError_t jacobi_epilogue_launch(const double* xs, int ldx, int l, int LP, const double* thr2, double* sigma,
                                  double* uhat_d, TU* uhat_p, TU* vhat_p, hipStream_t s);

// fp8.hip -- block-scaled OCP E4M3 copies of A (128 x 128 tile scales, shared by A8 and its transpose)
// and the FP8 MFMA product with an FP32 panel quantised per 128-row segment of each column.
hipError_t launch_to_fp8(const float* A, int64_t lda, int64_t m, int64_t n, uint8_t* A8, int64_t ld8, uint8_t* A8T,
                         int64_t ldT, float* scale, int* flag, hipStream_t s);
// The same codes and scales with A8 (m x n) and A8T (n x m) in the tiled layout of lowp_common.hpp
// (fp8_tiled_bytes(m, n) and fp8_tiled_bytes(n, m) bytes).
size_t fp8_tiled_bytes(int64_t rows, int64_t K);
hipError_t launch_to_fp8_tiled(const float* A, int64_t lda, int64_t m, int64_t n, uint8_t* A8, uint8_t* A8T,
                               float* scale, int* flag, hipStream_t s);
// lpgemm.hip -- products of a low-precision copy of A (kind 0: bf16, 1: E4M3 with tile scales, scale of row
// block rb and contraction block kb at sA[rb * s_row + kb * s_k]) with an FP32 panel converted once into
// FP64-accumulated Gram Y^T Y of an nc-column panel (FP32 or FP64), split-K partials as launch_nn (gram.hip);
// gram_tile_pairs(nc) workgroups per contraction range.
int gram_tile_pairs(int nc);
template <typename TI>
hipError_t launch_gram(const TI* Y, int64_t ld, int64_t K, int nc, double* out, int64_t ldo, int64_t part_stride,
                       int splits, hipStream_t s, const int* skip = nullptr);
// `scratch` (lp_scratch_bytes); output as launch_nn (split-K partials).
size_t lp_scratch_bytes(int kind, int64_t K, int ncols);
int lp_splits_used(int64_t K, int splits);
int64_t lp_row_workgroups(int kind, int64_t rows, int ncols);
int lp_resident_workgroups();
// tiled: A in the tiled layout of lowp_common.hpp (lda unused), else row-major.
hipError_t launch_nn_lp(int kind, bool tiled, const void* A, int64_t lda, const float* sA, int64_t s_row,
                        int64_t s_k, int64_t rows, int64_t K, const float* X, int64_t ldx, int ncols, void* scratch,
                        float* out, int64_t ldo, int64_t part_stride, int splits, hipStream_t s);

// mlp.hip -- the selector network (16 -> 64 -> 64 -> 40, FP32) and its training steps.
int mlp_param_count();
hipError_t launch_mlp_forward(const float* th, int B, const float* X, float* H1, float* H2, float* Z, hipStream_t s);
hipError_t launch_mlp_backward(const float* th, int B, const float* X, const float* H1, const float* H2,
                               const float* Z, const float* Y, const float* M, float* grad, float* loss,
                               float* scratch, hipStream_t s);
hipError_t launch_adam(float* th, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
// x[i] = log10(max(sigma[i+1] / sigma[0], 1e-12)) / 6 (i < 15), x[15] = log10(k) / 3.
hipError_t launch_sel_features(const double* sigma, int k, float* x, hipStream_t s);

// jacobi.hip
template <typename TU>
struct JacobiProblem {
  const double* R;     // the l x l matrix (column-major, leading dimension LP)
  double* sigma;
  double* uhat_d;
  TU* uhat_p;          // may be null
  TU* vhat_p;          // may be null
};
// Two independent problems of the same size (LP <= 128) in one launch, one workgroup each.
template <typename TU>
hipError_t launch_jacobi2(const JacobiProblem<TU>& a, const JacobiProblem<TU>& b, int l, int LP, double tol,
                          int max_sweeps, int* flags, hipStream_t s);
template <typename TU>
hipError_t launch_jacobi(const double* R, int l, int LP, double tol, int max_sweeps, double* sigma, double* uhat_d,
                         TU* uhat_p, TU* vhat_p, double* scratch, int* flags, hipStream_t s);

// lowp.hip -- bf16 copies of A (row-major and transposed, RNE, zero-padded to
// multiples of 128 columns).
hipError_t launch_to_bf16(const float* A, int64_t lda, int64_t m, int64_t n, uint16_t* A16, int64_t ld16,
                          uint16_t* A16T, int64_t ldT, int* flag, hipStream_t s);
// Both copies in the tiled layout of lowp_common.hpp (bf16_tiled_bytes(m, n) and bf16_tiled_bytes(n, m) bytes).
size_t bf16_tiled_bytes(int64_t rows, int64_t K);
hipError_t launch_to_bf16_tiled(const float* A, int64_t lda, int64_t m, int64_t n, uint16_t* A16, uint16_t* A16T,
                                int* flag, hipStream_t s);


// batched.hip
int batched_scratch_doubles_per_wg();
int batched_max_rank();
int batched_max_dim();
int batched_num_classes();
int batched_num_variants();
int batched_default_variant();
int batched_resident_per_cu();
// tiles: host array of batched_num_classes() variants (nullptr = default); blocks
// whose size class is outside class_mask are skipped.
hipError_t launch_batched(int nblk, const int* m, const int* n, const float* const* A, const int* lda, double eps,
                          int rank_cap, uint64_t seed, float* U, double* S, float* V, const int64_t* offU,
                          const int64_t* offV, int* rank, int* status, int* order, int* queue, double* scratch,
                          int nwg, const int* tiles, int class_mask, hipStream_t s);

// singlepass.hip -- small FP64 steps of the single-pass factorisations (column-major, op = transpose when set):
// out (M x N) = op(A) op(B) [+ out], column j divided by inv_scale[j] (0 where inv_scale[j] <= 0) when given.
template <typename TO>
hipError_t launch_small_gemm(int M, int N, int K, const double* A, int64_t lda, bool ta, const double* B, int64_t ldb,
                             bool tb, TO* out, int64_t ldo, bool acc, const double* inv_scale, hipStream_t s);
// X(i, j) /= a_i + b_j (zero where a_i + b_j <= cut_rel (a_0 + b_0)).
hipError_t launch_sylv_divide(double* X, int64_t ldx, int k1, int k2, const double* a, const double* b,
                              double cut_rel, hipStream_t s);
// x[i] <- bf16 rounding of x[i] (nearest, ties to even), stored in binary32.
hipError_t launch_round_bf16(float* x, int64_t n, hipStream_t s);
// out = in^T for an rows x cols FP64 matrix.
hipError_t launch_transpose64(const double* in, int64_t ldi, int rows, int cols, double* out, int64_t ldo,
                              hipStream_t s);
// out[j] = X(:, j) . Y(:, j).
hipError_t launch_coldot(const double* X, const double* Y, int64_t ld, int rows, int ncols, double* out,
                         hipStream_t s);

// idcur.hip -- k steps of column-pivoted QR of the l x N matrix whose columns are the rows of an N x l panel Y
// (l <= cpqr_max_rows()): pivots J, q vectors Q (l x k, leading dimension LQ), S = Q^T Y (k x N, row i at
// S + i * ldS); scratch nrm2, orig (N doubles each), blkmax/blkidx (cpqr_blocks(N) each), counter (one word).
int cpqr_max_rows();
int64_t cpqr_blocks(int64_t N);
template <typename T>
hipError_t launch_cpqr(const T* Y, int64_t ld, int64_t N, int l, int k, double* Q, int LQ, double* S, int64_t ldS,
                       double* nrm2, double* orig, double* blkmax, int* blkidx, unsigned* counter, int* J,
                       hipStream_t s);
// Z = S11^-1 S (k x N, row i at Z + i * ldZ) and/or X = Z^T (N x k row-major), S11 = S(:, J) into the k x k
// scratch S11 (leading dimension LK).
template <typename TX>
hipError_t launch_id_solve(const double* S, int64_t ldS, int64_t N, int k, const int* J, double* S11, int LK,
                           double* Z, int64_t ldZ, TX* X, int64_t ldx, hipStream_t s);
// out (m x k panel) = A(:, J); out (n x k FP64 panel) = A(I, :)^T.
template <typename T>
hipError_t launch_gather_cols(const T* A, int64_t lda, int64_t m, const int* J, int k, T* out, int64_t ldo,
                              hipStream_t s);
template <typename T>
hipError_t launch_gather_rows(const T* A, int64_t lda, int64_t n, const int* I, int k, double* out, int64_t ldo,
                              hipStream_t s);
// v[i] = 0 where v[i] <= rel v[0].
hipError_t launch_cut_small(double* v, int n, double rel, hipStream_t s);

// misc.hip
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s);
hipError_t launch_symmetrize(double* G, int64_t ldg, int l, hipStream_t s);
hipError_t launch_square(const double* in, double* out, int n, hipStream_t s);
template <typename T>
hipError_t launch_axpy_panel(T* Y, int64_t ldy, const T* X, int64_t ldx, int64_t rows, int ncols, T alpha,
                             hipStream_t s);
template <typename T>
hipError_t launch_colnorm(const T* X, int64_t ld, int64_t rows, int ncols, double* norms, hipStream_t s);
template <typename T>
hipError_t launch_frob2(const T* A, int64_t lda, int64_t m, int64_t n, double* partials, double* out, hipStream_t s);
template <typename TO>
hipError_t launch_rowmajor_to_panel(const double* src, int64_t rows, int64_t cols, int64_t ld_src, TO* dst,
                                    int64_t ld_dst, hipStream_t s);

// srht.hip -- the structured test matrix of Section 6 (signs, subset) and the sketch Y = A Omega.
int srht_max_n(int es);
template <typename T>
hipError_t launch_srht_setup(uint64_t seed, int n, int l, T* signs, int* subset, hipStream_t s);
template <typename T>
hipError_t launch_srht_sketch(const T* A, int64_t lda, int64_t m, int n, const T* signs, const int* subset, int l,
                              T* out, int64_t osr, int64_t osc, hipStream_t s);

// rsvd_api.hip: one fixed-rank factorisation (eps == 0, fixed p and q, no timing) in a caller-given
// workspace, with a plan built on the stack; RSVD_E_WORKSPACE when the description needs more than
// ws_bytes.  The same launch sequence as rsvd_plan + rsvd_factor with h_info == NULL.
int factor_in_workspace(const void* desc, void* ws, size_t ws_bytes, hipStream_t st, const void* A, int64_t lda,
                        const double* omega, void* U, int64_t ldu, double* S, void* V, int64_t ldv);

}  // namespace rsvd
