/*
 * rsvd_kernels.h -- kernel-level entry points of librsvd.so, exposed so each
 * building block of the randomized SVD can be checked on its own against a
 * CPU reference.  Same conventions as rsvd.h (device pointers d_*, work
 * enqueued on `stream`, RSVD_E_ARG before anything is enqueued).
 *
 * "Panel" layout: an r x c tall matrix P is stored column by column,
 * element (i, j) at P[j * ld + i] (the row-major storage of P^T).  The
 * library keeps Y = A Omega, Q, W, B^T and the other thin matrices this way.
 *
 * Precision codes: RSVD_F64 = inputs, arithmetic and output in FP64;
 * RSVD_F32 = FP32 inputs, FP32 MFMA, FP32 output; and for the products
 * only, 10 = FP32 inputs with FP64 MFMA accumulation and FP64 output (the
 * Gram matrices of the orthonormalisation).
 */
#ifndef RSVD_KERNELS_H_
#define RSVD_KERNELS_H_

#include "rsvd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RSVD_F32_ACC64 10

/*
 * d_out (panel, ld ldo >= rows) = A X for A rows x K row-major (lda >= K) and
 * X a K x ncols panel (ldx >= K): the product used for the sketch Y = A Omega,
 * the power step Y = A W (Section 8.1, Figure 5) and, with A a panel read as
 * its transpose, the Gram matrix Y^T Y of CholeskyQR.  1 <= ncols <= 1024.
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_product_nn(int32_t precision, int64_t rows, int64_t K, const void* d_A, int64_t lda,
                              const void* d_X, int64_t ldx, int32_t ncols, void* d_out, int64_t ldo,
                              void* stream);

/*
 * d_G (nc x nc FP64, column-major, ldg >= nc) = Y^T Y for Y a K x nc panel
 * (d_Y[c*ldy + i], precision RSVD_F32 or RSVD_F64, ldy >= K a multiple of 64,
 * 16-byte aligned): the Gram matrix of CholeskyQR (Section 2.3 allows any
 * unpivoted orthonormalisation; the library runs Cholesky on this FP64
 * Gram).  FP32 entries and their products are exact in FP64; the sum is
 * accumulated in FP64 on the FP64 MFMA.  Both triangles are written.
 * 1 <= nc <= 1024.  Caller owns all buffers; no allocation.
 * Errors: RSVD_E_ARG (sizes, alignment, precision), RSVD_E_HIP.
 */
rsvd_status rsvd_k_gram(int32_t precision, int64_t K, int32_t nc, const void* d_Y, int64_t ldy, double* d_G,
                        int64_t ldg, void* stream);

/*
 * d_out = A^T P for A K x N row-major (lda >= N) and P a K x ncols panel
 * (ldp >= K): the power step Z = A^T Q and the projection B^T = A^T Q
 * (Figure 5).  out_rowmajor = 0: d_out is an N x ncols panel (ldo >= N);
 * 1: d_out is N x ncols row-major (ldo >= ncols).
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_product_tn(int32_t precision, int64_t K, int64_t N, const void* d_A, int64_t lda,
                              const void* d_P, int64_t ldp, int32_t ncols, void* d_out, int64_t ldo,
                              int32_t out_rowmajor, void* stream);

/*
 * FP64 Cholesky of the l x l symmetric matrix d_G (column-major, ldg >= l):
 * G = R^T R with R upper triangular, R_jj > 0.  Writes d_Rinv (LP x LP FP64,
 * d_Rinv[c*LP + k] = R^-1(k, c), identity outside l x l) and d_R (LP x LP
 * FP64 row-major, identity outside l x l).  LP = l rounded up to 16.  Columns
 * whose pivot falls to <= tau_rel * G_jj are dropped (zero row of R, zero
 * column of R^-1) and counted in d_flags[1]; non-finite pivots in d_flags[0].
 * d_flags: 4 device ints, accumulated (not cleared).  l <= 128 runs in one
 * workgroup; larger l runs the blocked multi-workgroup form and needs
 * d_scratch (device, rsvd_k_scratch_bytes(l) bytes, caller-owned, contents
 * undefined afterwards); d_scratch may be NULL for l <= 128.
 * Errors: RSVD_E_ARG (l < 1 or l > 1024, or no scratch where one is needed),
 * RSVD_E_HIP.
 */
rsvd_status rsvd_k_cholesky(int32_t l, const double* d_G, int64_t ldg, double tau_rel, double* d_Rinv,
                            double* d_R, int32_t* d_flags, void* d_scratch, void* stream);

/*
 * SVD of X = R^T by one-sided Jacobi in FP64 (the small SVD of Stage B,
 * Section 3): d_R is LP x LP row-major (LP = l rounded up to 16), only its
 * leading l x l block read.  Writes d_sigma (LP values, descending, zeros
 * past l) and d_Uhat (LP x LP, column j of U_hat at d_Uhat[j*LP .. +LP)),
 * each column signed so that its entry of largest magnitude is positive.
 * A column whose norm is at most l u ||X||_F (numerically zero: X of lower
 * rank) takes no rotation and comes out as sigma = 0 with a zero column of
 * d_Uhat, as an exactly zero column does.
 * d_flags[2] counts a sweep limit reached before convergence, d_flags[3]
 * holds the largest sweep count.  l <= 128 runs in one workgroup with X in
 * LDS; larger l (up to 1024) runs block one-sided Jacobi over many
 * workgroups and needs d_scratch (rsvd_k_scratch_bytes(l) bytes; may be NULL
 * for l <= 128); that form runs up to 60 sweeps in one persistent launch
 * (its workgroups, at most 64, must all be resident: RSVD_E_HIP if the
 * device cannot hold them), stops after the first sweep without a rotation,
 * and never synchronises the host.  A grid barrier wait of that launch is
 * bounded at two seconds; running out of it counts in d_flags[0] and
 * d_flags[2].
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_small_svd(int32_t l, const double* d_R, double* d_sigma, double* d_Uhat, int32_t* d_flags,
                             void* d_scratch, void* stream);

/*
 * Bytes of device scratch that rsvd_k_cholesky and rsvd_k_small_svd need at
 * size l (0 for l <= 128).  Errors: RSVD_E_ARG (l < 1 or l > 1024, NULL
 * h_bytes).
 */
rsvd_status rsvd_k_scratch_bytes(int32_t l, size_t* h_bytes);

/*
 * Input preparation for the bf16 products: d_A16 (m x ld16 row-major bf16,
 * stored as uint16) = round-to-nearest-even bf16 of A (m x n FP32, lda >= n),
 * and d_A16T (n x ldT) = its transpose; columns past n (resp. m) are zero.
 * ld16 >= n and ldT >= m must be multiples of 128.  *d_flag (device int) gets
 * bit 0 set if A holds a NaN or an infinity.
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_convert_bf16(int64_t m, int64_t n, const float* d_A, int64_t lda, uint16_t* d_A16, int64_t ld16,
                                uint16_t* d_A16T, int64_t ldT, int32_t* d_flag, void* stream);

/*
 * d_out (panel, ldo >= rows, FP32) = A16 X for A16 rows x K bf16 as written by
 * rsvd_k_convert_bf16 (lda a multiple of 128, zero past K) and X a K x ncols
 * FP32 panel (X[c*ldx + k], ldx >= K) rounded to bf16 (nearest even) by a
 * conversion pass into d_scratch (device, 256-byte aligned,
 * rsvd_k_lp_scratch_bytes(RSVD_BF16, K, ncols) bytes); bf16 MFMA with FP32
 * accumulation.  1 <= ncols <= 1024.
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_product_bf16(int64_t rows, int64_t K, const uint16_t* d_A16, int64_t lda, const float* d_X,
                                int64_t ldx, int32_t ncols, float* d_out, int64_t ldo, void* d_scratch,
                                void* stream);

/*
 * Bytes of the thin-operand scratch of rsvd_k_product_bf16 (dtype RSVD_BF16)
 * and rsvd_k_product_fp8 (RSVD_FP8_E4M3) for K x ncols.
 * Errors: RSVD_E_ARG.
 */
rsvd_status rsvd_k_lp_scratch_bytes(int32_t dtype, int64_t K, int32_t ncols, size_t* h_bytes);

/*
 * Input preparation for the FP8 products (OCP E4M3: bias 7, 3 mantissa bits,
 * largest finite 448, round to nearest even, saturating): for every 128 x 128
 * tile (ti, tj) of A (m x n FP32, lda >= n), scale[ti * (ld8/128) + tj] = 2^e
 * with e the least integer such that max|tile| <= 448 2^e (1 for a zero
 * tile), d_A8 (m x ld8 bytes, row-major) = E4M3 codes of A / scale and d_A8T
 * (n x ldT) the same codes transposed; zeros past n (resp. m).  ld8 >= n and
 * ldT >= m multiples of 128; d_A8, d_A8T 16-byte aligned.  *d_flag gets bit 0
 * set if A holds a NaN or an infinity.  (The block-scaled format of the
 * precision growth; tiles serve both orientations.)
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_convert_fp8(int64_t m, int64_t n, const float* d_A, int64_t lda, uint8_t* d_A8, int64_t ld8,
                               uint8_t* d_A8T, int64_t ldT, float* d_scale, int32_t* d_flag, void* stream);

/*
 * d_out (panel, ldo >= rows, FP32) = A X for A (rows x K) given as E4M3 codes
 * d_A8 (lda a multiple of 128, zero past K) with the scale of row block rb
 * (128 rows) and contraction block kb (128) at d_scale[rb * s_row + kb * s_k],
 * and X a K x ncols FP32 panel (X[c*ldx + k], ldx >= K) quantised by a
 * conversion pass into d_scratch (device, 256-byte aligned,
 * rsvd_k_lp_scratch_bytes(RSVD_FP8_E4M3, K, ncols) bytes) to E4M3 with one
 * power-of-two scale per 128-row segment of each column.  FP8 MFMA with FP32
 * accumulation; each 128-wide block's partial product is scaled and added.
 * 1 <= ncols <= 1024.
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_product_fp8(int64_t rows, int64_t K, const uint8_t* d_A8, int64_t lda, const float* d_scale,
                               int64_t s_row, int64_t s_k, const float* d_X, int64_t ldx, int32_t ncols,
                               float* d_out, int64_t ldo, void* d_scratch, void* stream);

/*
 * The structured test matrix of Section 6 in real form and the sketch with it
 * (the draw and the transform that rsvd_factor runs under RSVD_SKETCH_SRHT):
 *   d_signs  (device, n entries of prec) <- d_i in {+1, -1}
 *   d_subset (device, l int32)           <- s_0 .. s_{l-1}, distinct, < N
 *   d_Y      (device, m x l row-major, ldy >= l, prec) <- A Omega,
 *            Omega = (D H_N S / sqrt(N))[:n, :], N = 2^ceil(log2 n)
 * for A (m x n row-major, lda >= n, prec = RSVD_F32 or RSVD_F64).  The draw
 * (Philox4x32-10, key = seed, stream 10) is the one documented with
 * RSVD_SKETCH_SRHT in rsvd.h.  1 <= l <= min(1024, N); n <= 32768 (F32) or
 * 16384 (F64).  Arithmetic in prec (the transform adds and subtracts only).
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_k_srht_sketch(int32_t prec, int64_t m, int64_t n, const void* d_A, int64_t lda, int32_t l,
                               uint64_t seed, void* d_signs, int32_t* d_subset, void* d_Y, int64_t ldy,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_KERNELS_H_ */
