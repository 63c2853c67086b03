/*
 * rsvd.h -- C ABI of the MI355X (gfx950) randomized range finder and
 * randomized SVD.
 *
 * The method is the two-stage scheme of P.-G. Martinsson, "Randomized
 * methods for matrix computations": Stage A finds an orthonormal Q with
 * A ~= Q Q^T A from a Gaussian sketch Y = A Omega, refined by q power steps
 * with re-orthonormalisation after every application of A or A^T (Section
 * 8.1, Figure 5); Stage B forms B = Q^T A, the SVD B = U_hat D V^T, and
 * U = Q U_hat (Section 3).  An optional a-posteriori certificate (Section
 * 14, built on the Gaussian-probe lemma of Section 13) judges the result and
 * triggers the blocked adaptive range finder of Figure 12 (Section 12.3) when
 * the tolerance is missed.
 *
 * Conventions shared by every entry point
 *   - Matrices are ROW-MAJOR with an explicit leading dimension (elements).
 *   - Pointers named d_* are device pointers; h_* are host pointers.
 *   - The caller owns every buffer (A, outputs, workspace).  The library never
 *     allocates device memory; all scratch comes from the workspace handed to
 *     rsvd_plan.  A is never written.
 *   - Work is enqueued asynchronously on the plan's HIP stream (passed as a
 *     void* holding a hipStream_t; NULL = the default stream).  An entry point
 *     synchronises that stream only where its comment says so.
 *   - Argument errors are detected on the host before anything is enqueued and
 *     return RSVD_E_ARG; nothing is printed unless the environment variable
 *     RSVD_LOG is set.
 */
#ifndef RSVD_H_
#define RSVD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSVD_OK = 0,
  RSVD_NOT_CERTIFIED = 1,   /* factors written; the certificate still exceeds eps at max_rank */
  RSVD_E_ARG = -1,          /* invalid argument (host-side check, nothing enqueued)          */
  RSVD_E_WORKSPACE = -2,    /* workspace null or smaller than rsvd_workspace_size            */
  RSVD_E_HIP = -3,          /* a HIP runtime call failed                                       */
  RSVD_E_NONFINITE = -4,    /* NaN or Inf met in the computation; outputs undefined            */
  RSVD_E_UNSUPPORTED = -5   /* valid but not built (e.g. a dtype combination)                  */
} rsvd_status;

typedef enum {
  RSVD_F64 = 0,        /* IEEE binary64                                                   */
  RSVD_F32 = 1,        /* IEEE binary32                                                   */
  RSVD_BF16 = 2,       /* bfloat16, round-to-nearest-even from FP32                       */
  RSVD_FP8_E4M3 = 3    /* OCP FP8 E4M3 with one power-of-two scale per 128x128 tile of A  */
} rsvd_dtype;

/* rsvd_desc.flags */
#define RSVD_RETURN_RANK_L 0x1u  /* return all l = k+p columns instead of the k leading ones   */
#define RSVD_TIMING        0x2u  /* record per-stage HIP events; rsvd_info.stage_ms filled    */
#define RSVD_SKETCH_SRHT   0x4u  /* first sketch with the structured test matrix (see below)  */
#define RSVD_NYSTROM       0x8u  /* Nystrom eigendecomposition of a psd matrix (see below)     */
#define RSVD_SINGLE_PASS   0x10u /* single-pass SVD of a general matrix (see below)            */
#define RSVD_SINGLE_PASS_SYM 0x20u /* single-pass EVD of a symmetric matrix (see below)        */
#define RSVD_ID_CUR        0x40u /* plan for rsvd_row_id / rsvd_cur (see there)                */

/*
 * Problem description.
 *   m, n        shape of A (1 <= k+p <= min(m, n)).
 *   k, p        target rank and oversampling; l = k + p columns are sketched
 *               (Section 4; p = 10 is the paper's usual choice).
 *   q           number of power steps of Figure 5 (q >= 0).
 *               p = q = -1 selects the learned selector: before each
 *               factorisation a 16-column probe sketch and the network set
 *               with rsvd_selector_set choose (p, q) from the grid below
 *               (reported in rsvd_info.p_used / q_used).
 *   seed        seeds the Gaussian test matrix.  Entry (i, j) of every Gaussian
 *               matrix the library draws is a function of (seed, stream, i, j)
 *               only: Philox4x32-10 (Salmon et al., SC'11) with key = seed,
 *               counter = (i/2, j, stream, 0), then Box-Muller on two 53-bit
 *               uniforms (row parity picks cos or sin).  Streams: 4 = Omega and
 *               the fallback blocks that extend it, 6 = certificate probes.
 *   a_dtype     RSVD_F64 or RSVD_F32: dtype of A, U and V.
 *   sketch_dtype, proj_dtype
 *               operand precision of the products with A in Stage A (A*Omega,
 *               A^T*Q, A*W) and of the projection B = Q^T A.  F64 requires
 *               a_dtype F64; F32 requires a_dtype F32 (F32 MFMA, FP32
 *               accumulation); BF16 and FP8_E4M3 require a_dtype F32 and
 *               accumulate in FP32.  The Gram matrices of the
 *               orthonormalisation are accumulated in FP64 and factored in
 *               FP64; the small SVD of B always runs in FP64.
 *   eps         0: fixed rank k.  > 0: certify ||A - U D V^T|| <= eps * D(1)
 *               with the Section 14 certificate and grow the basis with the
 *               blocked range finder of Figure 12 until it holds.
 *   n_probe     r, number of certificate probes (0 -> 10).
 *   est_power   s >= 0: the certificate is taken of (T T^T)^s T, T = A - U D V^T,
 *               and its (2s+1)-th root returned (0 = the paper's form).
 *   fallback_block  b, columns added per growth step (0 -> 32).
 *   max_rank    when eps > 0: largest basis the fallback may grow to, and the
 *               column capacity U and V must have (>= k+p; 0 -> k+p, i.e. no
 *               growth).
 *   flags       RSVD_RETURN_RANK_L | RSVD_TIMING | RSVD_SKETCH_SRHT | RSVD_NYSTROM.
 *
 * RSVD_SKETCH_SRHT (Section 6; Section 14, item (1)): the first sketch is
 * Y = A Omega with the structured test matrix Omega = D F S in real form:
 * N = 2^ceil(log2 n) (A's rows zero-padded to N), D = diag of random signs,
 * F = H_N / sqrt(N) with the Walsh-Hadamard matrix H_N(i, k) =
 * (-1)^popcount(i & k), S = k+p distinct columns of the N x N identity
 * drawn by a seeded Fisher-Yates shuffle (Philox4x32-10, key = seed, stream
 * 10: sign i = lowest bit of word i mod 4 of counter (i div 4, 0, 10, 0);
 * shuffle step j swaps entries j and j + floor(u_j (N - j) / 2^32) of the
 * identity permutation, u_j = word j mod 4 of counter (j div 4, 1, 10, 0)).
 * It is computed by a fast transform in one pass over A (O(m n log l));
 * the power steps, Stage B, the certificate and the fallback (Gaussian
 * blocks, stream 4, continuing at column k+p) are unchanged.  Needs
 * sketch_dtype == a_dtype, n <= 32768 (F32) or 16384 (F64), fixed p and q
 * (no selector); RSVD_E_ARG otherwise.
 *
 * RSVD_NYSTROM (Section 9 and its figure): for a symmetric positive
 * semidefinite A (m == n), the eigendecomposition A ~= U diag(S) U^T by the
 * Nystrom method: Q from Stage A (q = 0 is the figure as printed; q >= 1
 * adds Figure 5's power steps), B1 = A Q (operands in proj_dtype), B2 =
 * Q^T B1 accumulated in FP64 and made exactly symmetric, B2 = C^T C
 * (Cholesky, pivots at or below (k+p) u times the diagonal dropped and
 * counted in dropped_cols, which counts nothing else here), F = B1 C^-1, the SVD F = U Sigma W^T (FP64, as Stage B),
 * S = Sigma^2 (descending, >= 0).  d_U gets U (n x r), d_V (if not NULL)
 * the same U, so that U diag(S) V^T is the approximation.  Needs m == n,
 * eps == 0 and fixed p, q (RSVD_E_ARG otherwise); A's symmetry is assumed,
 * not checked.
 *
 * RSVD_SINGLE_PASS (Section 5.2 and its figure): the SVD of a general A from
 * one pass over it.  G_c (n x l, stream 4, or d_Omega) and G_r (m x l, stream
 * 11) Gaussian; Y_c = A G_c and Y_r = A^T G_r; Q_c, Q_r = the k dominant left
 * singular vectors of Y_c, Y_r (FP64 small SVD, as Stage B); the k x k core C
 * = the least-squares solution of the joint system (G_r^T Q_c) C = Y_r^T Q_r,
 * C (Q_r^T G_c) = Q_c^T Y_c (both residuals weighted equally; products
 * accumulated in FP64; solved through its normal equations, entries of C along
 * directions that neither equation set determines are zero); C = U_hat D
 * V_hat^T; U = Q_c U_hat, V = Q_r V_hat.  Each pair (u_j, v_j) is unique up
 * to a common sign.
 *
 * RSVD_SINGLE_PASS_SYM (Section 5.1 and its figure): the EVD A ~= U diag(S)
 * U^T of a symmetric A (m == n; symmetry assumed, not checked): G (n x l,
 * stream 4, or d_Omega), Y = A G, Q = the k dominant left singular vectors of
 * Y, C = the least-squares solution of C (Q^T G) = Q^T Y over symmetric C, C =
 * U_hat D U_hat^T, U = Q U_hat.  S holds the signed eigenvalues ordered by
 * decreasing magnitude; d_V (if not NULL) gets U.
 *
 * Both need q == 0, eps == 0, fixed p (no selector), sketch_dtype ==
 * proj_dtype equal to a_dtype or RSVD_BF16 (then G_c and G_r are rounded to
 * bf16 values before use, so the equations see the matrices the sketches
 * were formed with; no projection pass) and neither
 * RSVD_RETURN_RANK_L, RSVD_SKETCH_SRHT nor RSVD_NYSTROM (RSVD_E_ARG
 * otherwise); the two flags exclude each other.
 */
typedef struct {
  int64_t m, n;
  int32_t k, p, q;
  int32_t a_dtype, sketch_dtype, proj_dtype;
  uint64_t seed;
  double eps;
  int32_t n_probe, est_power;
  int32_t fallback_block, max_rank;
  uint32_t flags;
  uint32_t reserved_;
} rsvd_desc;

/* Filled by rsvd_factor when h_info is not NULL (that call then synchronises
 * the plan's stream). */
typedef struct {
  int32_t p_used, q_used;
  int32_t rank_out;        /* columns written to U and V                              */
  int32_t fallback_steps;  /* growth steps of the blocked range finder               */
  int32_t reserved0;       /* always 0                                                */
  int32_t status;          /* same value as the return code                          */
  double err_bound;        /* certificate value (absolute); 0 when eps == 0           */
  double sigma1;           /* D(1)                                                    */
  float stage_ms[8];       /* with RSVD_TIMING: sketch, power, project, small SVD,
                              lift, certificate, fallback, total                     */
  float nn_ms, tn_ms;      /* with RSVD_TIMING: summed durations of the products A*X
                              and A^T*X (HIP events around each launch)              */
  int32_t nn_launches, tn_launches;
  int32_t jacobi_sweeps;   /* sweeps of the small SVD                                 */
  int32_t dropped_cols;    /* numerically dependent columns met by CholeskyQR: a Gram
                              pivot <= l u^2 G_jj (u the unit roundoff of the data)
                              gives a zero column of the basis instead of a failure
                              (no retry), so for a rank-deficient A the basis spans
                              its numerical range and the columns of U and V past
                              that rank are zero, with zero singular values          */
  double frob_residual;    /* after a fallback: sqrt(||A||_F^2 - ||B||_F^2) (Section 12.4
                              downdating) of the grown basis; -1 otherwise            */
} rsvd_info;

typedef struct rsvd_plan_s* rsvd_plan_t;

/*
 * Learned (p, q) selector.  The paper fixes p by a rule of thumb (Section 4:
 * p = 10) and q by experience (Section 8: q = 1 or 2); the selector picks
 * them per matrix for a tolerance instead.
 *   Probe: Y16 = A G16 with 16 Gaussian columns of stream 5; sigma_1 >= ..
 *   >= sigma_16 its singular values (FP64 CholeskyQR + Jacobi).
 *   Input x (16 floats): x_i = log10(max(sigma_{i+1} / sigma_1, 1e-12)) / 6
 *   for i = 0..14, x_15 = log10(k) / 3.
 *   Network: 16 -> 64 (ReLU) -> 64 (ReLU) -> 40 logits, FP32; parameters in
 *   one flat vector of RSVD_MLP_NPARAM floats: W1 (64 x 16 row-major), b1
 *   (64), W2 (64 x 64), b2 (64), W3 (40 x 64), b3 (40).
 *   Output o = 8 * iq + ip is the predicted probability (logistic of the
 *   logit) that p = RSVD_SEL_P[ip], q = iq (0..4) meets the tolerance
 *   without growth.
 *   Decision: among grid points with k + p <= min(m, n, 1024) and
 *   probability P >= tau, the one of least expected time c(p, q) (2 - P) (a
 *   miss is taken to double the time through the fallback); if none, the
 *   most probable one.  Modelled time (ms) at l = k + p:
 *     c = 0.081 + (2q+2) 2 m n l 20.9e-12 + (2q+1) 0.104 max(l/128, 1)^1.5
 *         + 1.08 (l/95)^1.5
 *   (passes over A, CholeskyQR passes and the Stage B Jacobi, fitted by
 *   non-negative least squares to 120 measured MI355X timings of the plain
 *   method on items of the selector's training distribution; median relative
 *   error 9 %).
 */
#define RSVD_MLP_IN 16
#define RSVD_MLP_HIDDEN 64
#define RSVD_MLP_OUT 40
#define RSVD_MLP_NPARAM 7848
#define RSVD_SEL_NP 8
#define RSVD_SEL_NQ 5
#define RSVD_SEL_P_INIT {0, 5, 10, 20, 40, 80, 160, 320}

/* Human-readable name of a status code (static string). */
const char* rsvd_status_str(int status);

/*
 * Bytes of device workspace rsvd_plan needs for this description.
 * Errors: RSVD_E_ARG for an invalid description or null h_bytes.
 */
rsvd_status rsvd_workspace_size(const rsvd_desc* d, size_t* h_bytes);

/*
 * Validate the description, carve the caller's workspace (d_ws, ws_bytes,
 * 256-byte aligned) and bind the plan to a HIP stream.  The plan is a host
 * object owned by the library until rsvd_destroy; it is bound to one stream
 * and must not be used from two host threads at once.  Workspace contents are
 * undefined between calls.  Enqueues nothing.
 * Errors: RSVD_E_ARG, RSVD_E_WORKSPACE, RSVD_E_UNSUPPORTED, RSVD_E_HIP.
 */
rsvd_status rsvd_plan(const rsvd_desc* d, void* d_ws, size_t ws_bytes, void* stream,
                      rsvd_plan_t* h_out);

/*
 * Randomized SVD of A (Figure 5 of the paper, then Section 3's Stage B):
 *   d_A     m x n, a_dtype, row-major with leading dimension lda >= n.
 *   d_Omega optional n x (k+p) FP64 test matrix, row-major, leading
 *           dimension k+p; NULL draws it from the seed.  (A given Omega lets a
 *           caller reproduce a run with an external generator.)
 *   d_U     m x r output, a_dtype, row-major, ldu >= r.
 *   d_S     r singular values, FP64, descending.
 *   d_V     n x r output, a_dtype, row-major, ldv >= r (the paper's V, not V^T).
 *   r = k, or k+p with RSVD_RETURN_RANK_L, or (eps > 0) up to max_rank: the
 *   number written is rank_out.  Columns beyond rank_out are untouched.
 *   Columns are signed so that the entry of largest magnitude of each column
 *   of U_hat (the small SVD's left vectors) is positive.
 * Asynchronous when eps == 0 and h_info == NULL.  With eps > 0 the host reads
 * the certificate after the fixed-rank pass and once per growth step (stream
 * synchronised); ldu and ldv must then be >= max(k or k+p, max_rank).
 * Certificate (eps > 0): r = n_probe Gaussian vectors g_i (stream 6),
 * bound = 10 sqrt(2/pi) max_i ||(A - U D V^T) g_i|| (alpha = 1/10), which
 * exceeds ||A - U D V^T|| with probability at most 10^-r; accepted when
 * bound <= eps * D(1).  Otherwise the basis grows by fallback_block columns
 * per step (Figure 12, residual applied implicitly, each new block projected
 * against the basis twice) until the bound holds or max_rank is reached; all
 * columns of the grown basis are then returned (rank_out = its width).
 * Errors: RSVD_E_ARG (nothing enqueued), RSVD_E_HIP, RSVD_E_NONFINITE;
 * RSVD_NOT_CERTIFIED (> 0) when eps is missed at max_rank.
 * Reported only when h_info != NULL or eps > 0: device-side conditions
 * (non-finite values) need a synchronisation to be seen.  CholeskyQR never
 * fails on rank deficiency: dependent columns are dropped and counted in
 * rsvd_info.dropped_cols.
 */
rsvd_status rsvd_factor(rsvd_plan_t plan, const void* d_A, int64_t lda, const double* d_Omega,
                        void* d_U, int64_t ldu, double* d_S, void* d_V, int64_t ldv,
                        rsvd_info* h_info);

/*
 * Randomized row interpolative decomposition (Section 10.4, the figure with
 * q power steps): A ~= X A(I_s, :) with I_s k row indices and X (m x k) the
 * interpolation matrix (X(I_s, :) = I_k).  The plan's description must carry
 * RSVD_ID_CUR, k + p <= 128, eps == 0, sketch_dtype == proj_dtype == a_dtype
 * (RSVD_E_ARG otherwise).  The sample is Y = A G (G: n x (k+p) Gaussian,
 * stream 4, or d_Omega), and for q >= 1 Y = A orth(A^T orth(Y)) q times
 * (Figure 5's last sketch before its final orthonormalisation: the span of
 * (A A^T)^q A G, kept stable); [I_s, X] = the row ID of Y by k steps of
 * column-pivoted QR of Y^T (largest residual norm first, lowest index on
 * ties; FP64), X = (S11^-1 S)^T.  d_Is: k int32 (device), d_X: m x k
 * row-major (ldx >= k) in a_dtype.  Asynchronous when h_info == NULL.
 */
rsvd_status rsvd_row_id(rsvd_plan_t plan, const void* d_A, int64_t lda, const double* d_Omega,
                        int32_t* d_Is, void* d_X, int64_t ldx, rsvd_info* h_info);

/*
 * Randomized CUR (Section 11 and its figure): A ~= A(:, J_s) U A(I_s, :).
 * Plan as for rsvd_row_id.  The row sample Y (k+p x n) is the sample above
 * for A^T (G: m x (k+p), stream 4); [J_s, Z] = the column ID of Y (k steps
 * of column-pivoted QR, Z = S11^-1 S); I_s = the k pivots of the
 * column-pivoted QR of A(:, J_s)^T; U (k x k) = the least-squares solution
 * of U A(I_s, :) = Z through its normal equations (R = A(I_s, :), R R^T = V
 * diag(lambda) V^T by Jacobi, eigenvalues at or below k u lambda_1 dropped:
 * the minimum-norm solution where R is rank deficient).  d_Js, d_Is: k
 * int32 each (device); d_U: k x k row-major FP64 (ldu >= k).
 */
rsvd_status rsvd_cur(rsvd_plan_t plan, const void* d_A, int64_t lda, int32_t* d_Js, double* d_U, int64_t ldu,
                     int32_t* d_Is, rsvd_info* h_info);

/* Release a plan (host memory and events only; the workspace stays the
 * caller's). NULL is ignored. */
void rsvd_destroy(rsvd_plan_t plan);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * fixed-rank factorisation of rsvd_factor (eps == 0, h_info == NULL) with no
 * plan and no caller workspace.  Arguments d_A .. ldv as for rsvd_factor;
 * stream is a hipStream_t.  The workspace is one library-held device array of
 * RSVD_NOALLOC_WORKSPACE_BYTES per device (taken at the first call on that
 * device, held until the process ends); the call allocates nothing and is
 * asynchronous (enqueues kernels and device-to-device copies only).
 * Every call on one device shares that device's array: calls that overlap
 * on one device (two streams, two host threads) race and give undefined
 * results.  The array keeps the last call's contents; nothing in it needs
 * to start at zero.
 * Limits: fixed p, q >= 0 (no selector), eps == 0 (no certificate or
 * growth), no RSVD_TIMING, and rsvd_workspace_size(d) at most
 * RSVD_NOALLOC_WORKSPACE_BYTES (for instance 2000 x 2000 in FP64 at
 * k + p = 30 needs 6 MiB, 4000 x 3000 in FP32 at k + p = 128 needs 35 MiB,
 * 20000 x 20000 in FP32 at k + p = 110 needs 308 MiB and is refused; the
 * low-precision paths only for small A, whose converted copies live in the
 * workspace).  Non-finite input is not reported (use
 * rsvd_factor with h_info for that).
 * Errors: RSVD_E_ARG (as rsvd_factor, or a limit above), RSVD_E_WORKSPACE
 * (the description needs more than the array), RSVD_E_UNSUPPORTED (dtype
 * combination, or device ordinal >= 64), RSVD_E_HIP.
 */
#define RSVD_NOALLOC_WORKSPACE_BYTES (64ull << 20)
rsvd_status rsvd_factor_noalloc(const rsvd_desc* d, const void* d_A, int64_t lda, const double* d_Omega,
                                void* d_U, int64_t ldu, double* d_S, void* d_V, int64_t ldv, void* stream);

/*
 * Attach selector parameters to a plan made with p = q = -1: d_theta
 * (device, RSVD_MLP_NPARAM floats, caller-owned, must stay valid while the
 * plan is used) and the probability threshold tau in (0, 1).
 * Errors: RSVD_E_ARG (null plan or theta, tau outside (0, 1), plan not in
 * selector mode).
 */
rsvd_status rsvd_selector_set(rsvd_plan_t plan, const float* d_theta, float tau);

/*
 * The probe of the selector on its own: d_sigma16 (device, 16 doubles) =
 * singular values of A G16, descending, and d_x (device, 16 floats, may be
 * NULL) = the network input for the plan's k.  Uses the plan's workspace and
 * stream (any plan whose l = k + p is >= 16, or a selector-mode plan).
 * Errors: RSVD_E_ARG (null pointers, lda < n, plan too narrow), RSVD_E_HIP.
 */
rsvd_status rsvd_probe_sigma(rsvd_plan_t plan, const void* d_A, int64_t lda, double* d_sigma16, float* d_x);

/*
 * Certificates of every prefix of one Stage A basis (the labels of the
 * selector): Stage A of Figure 5 with the plan's l = k + p columns and q
 * power steps gives Q (m x l); for each width w = h_widths[i] (1 <= w <= l)
 * h_bounds[i] = 10 sqrt(2/pi) max_j ||(I - Q_w Q_w^T) A g_j|| with Q_w the
 * first w columns of Q and g_j the n_probe certificate probes (stream 6).
 * Because the test-matrix columns are prefix-stable and CholeskyQR keeps
 * prefixes, Q_w is (up to rounding) the basis the plain method builds with w
 * columns, so h_bounds[i] is the Section 14 certificate of the rank-w result
 * of the plain method.  The plan needs eps > 0 (for the probe buffers) and a
 * fixed p, q >= 0.  Synchronises the stream.
 * Errors: RSVD_E_ARG, RSVD_E_HIP, RSVD_E_NONFINITE.
 */
rsvd_status rsvd_prefix_bounds(rsvd_plan_t plan, const void* d_A, int64_t lda, int32_t n_widths,
                               const int32_t* h_widths, double* h_bounds);

/*
 * Selector network, forward pass over a batch: d_X (batch x 16), outputs the
 * hidden activations after ReLU d_H1, d_H2 (batch x 64) and the logits d_Z
 * (batch x 40), all FP32 row-major, device.  Sums in a fixed order.
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_mlp_forward(const float* d_theta, int32_t batch, const float* d_X, float* d_H1, float* d_H2,
                             float* d_Z, void* stream);

/*
 * Backward pass of the mean binary cross-entropy with logits over the
 * entries whose mask d_M (batch x 40, 0 or 1) is 1, labels d_Y (batch x 40):
 * d_grad (RSVD_MLP_NPARAM floats) = gradient with respect to theta, in the
 * parameter layout; d_loss[0] = the loss, d_loss[1] = the number of masked-in
 * entries.  d_X, d_H1, d_H2, d_Z as left by rsvd_mlp_forward.  d_scratch:
 * batch * 168 floats of device scratch.  Deterministic (fixed-order sums).
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_mlp_backward(const float* d_theta, int32_t batch, const float* d_X, const float* d_H1,
                              const float* d_H2, const float* d_Z, const float* d_Y, const float* d_M,
                              float* d_grad, float* d_loss, float* d_scratch, void* stream);

/*
 * One Adam step (Kingma and Ba, 2015) on n parameters, step >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_mlp_adam(float* d_theta, const float* d_grad, float* d_m, float* d_v, int32_t n, float lr,
                          float beta1, float beta2, float eps, int32_t step, void* stream);

/*
 * Batched compression of many independent blocks to a relative tolerance, in
 * one persistent launch (the given-tolerance problem of Sections 12-14 per
 * block).  Block b (0 <= b < nblk) is d_A[b] (device pointer), m_b x n_b FP32
 * row-major with leading dimension lda_b >= n_b, 16 <= m_b, n_b <= 512.  Per
 * block: l0 = 16 Gaussian columns, Q = orth(A Omega) and B = Q^T A in FP64
 * accumulation; certificate of the pair (Q, B) with 10 probes (Section 14);
 * while 10 sqrt(2/pi) max_i ||(A - QB) g_i|| > eps sigma_hat_1 / 2 the basis
 * grows by 8 columns (Figure 12, Omega's continuation, projected twice);
 * then the SVD of B and the singular values > eps sigma_hat_1 / 2 are kept,
 * so that ||A - U S V^T|| <= eps sigma_hat_1 with the certificate's
 * probability.  sigma_hat_1 = largest singular value of the first B.
 * Random streams per block: 16 b + 4 (Omega), 16 b + 6 (probes), key = seed.
 * Outputs (device): U_b at d_U + d_offU[b], m_b x rank_cap row-major (ld =
 * rank_cap); V_b at d_V + d_offV[b], n_b x rank_cap; S_b at d_S + b*rank_cap;
 * d_rank[b] = columns kept; d_status[b] = 0 certified, 1 not certified at the
 * rank cap, -1 invalid block shape, -4 non-finite entries.
 * eps in (0, 1); 16 <= rank_cap <= 64.  n_workgroups = persistent workgroups
 * (0 = as many as are resident at once on the device).  Blocks are taken
 * largest first from an atomic queue.  The products with the block run on the
 * FP64 MFMA in wave tiles whose shape is chosen per size class: h_tiles (host,
 * RSVD_BATCHED_CLASSES entries, or NULL for the default) gives the variant
 * (0 .. RSVD_BATCHED_TILE_VARIANTS-1) for blocks with max(m_b, n_b) in
 * (0,128], (128,256], (256,384], (384,512]; variant v takes 1 + (v & 1)
 * 16-row tiles and 1 + ((v >> 1) & 1) 16-column tiles per wave task with
 * 2 << ((v >> 2) & 1) k-slices in flight.  All variants give bit-identical
 * outputs; rsvd_batched_autotune picks the fastest.  Fully asynchronous; no
 * host synchronisation; capturable.
 * Workspace: rsvd_batched_workspace_size(nblk, n_workgroups).
 * Errors: RSVD_E_ARG (also a variant out of range), RSVD_E_WORKSPACE,
 * RSVD_E_HIP.
 */
#define RSVD_BATCHED_CLASSES 4
#define RSVD_BATCHED_TILE_VARIANTS 8
rsvd_status rsvd_batched_workspace_size(int32_t nblk, int32_t n_workgroups, size_t* h_bytes);
rsvd_status rsvd_batched(int32_t nblk, const int32_t* d_m, const int32_t* d_n, const float* const* d_A,
                         const int32_t* d_lda, double eps, int32_t rank_cap, uint64_t seed, float* d_U, double* d_S,
                         float* d_V, const int64_t* d_offU, const int64_t* d_offV, int32_t* d_rank,
                         int32_t* d_status, int32_t n_workgroups, const int32_t* h_tiles, void* d_ws,
                         size_t ws_bytes, void* stream);

/*
 * Tile autotuner of rsvd_batched (same arguments, minus h_tiles).  For every
 * size class that holds blocks it times each tile variant with HIP events
 * (one warm-up and two timed launches in which only that class's blocks are
 * compressed) and writes the fastest variant per class to h_tiles_out
 * (RSVD_BATCHED_CLASSES entries; the default for empty classes).  h_ms_out
 * (optional, RSVD_BATCHED_CLASSES x RSVD_BATCHED_TILE_VARIANTS, row-major)
 * receives the mean milliseconds per launch (0 for empty classes).
 * Synchronises `stream`; not capturable.  The outputs hold partial results
 * afterwards: run rsvd_batched (or a graph) with the chosen tiles.
 * Errors: as rsvd_batched.
 */
rsvd_status rsvd_batched_autotune(int32_t nblk, const int32_t* d_m, const int32_t* d_n, const float* const* d_A,
                                  const int32_t* d_lda, double eps, int32_t rank_cap, uint64_t seed, float* d_U,
                                  double* d_S, float* d_V, const int64_t* d_offU, const int64_t* d_offV,
                                  int32_t* d_rank, int32_t* d_status, int32_t n_workgroups, void* d_ws,
                                  size_t ws_bytes, void* stream, int32_t* h_tiles_out, float* h_ms_out);

/*
 * Capture one rsvd_batched call (same arguments, the tile table included) on
 * `stream` (not the NULL stream) into a HIP graph and instantiate it; rsvd_graph_launch replays it
 * on any stream (the buffers named at capture are reused).  The sequence
 * contains kernels only (no memset nodes).
 * Errors: RSVD_E_ARG, RSVD_E_WORKSPACE, RSVD_E_HIP.
 */
typedef struct rsvd_graph_s* rsvd_graph_t;
rsvd_status rsvd_batched_graph_create(int32_t nblk, const int32_t* d_m, const int32_t* d_n,
                                      const float* const* d_A, const int32_t* d_lda, double eps, int32_t rank_cap,
                                      uint64_t seed, float* d_U, double* d_S, float* d_V, const int64_t* d_offU,
                                      const int64_t* d_offV, int32_t* d_rank, int32_t* d_status,
                                      int32_t n_workgroups, const int32_t* h_tiles, void* d_ws, size_t ws_bytes,
                                      void* stream, rsvd_graph_t* h_out);
rsvd_status rsvd_graph_launch(rsvd_graph_t graph, void* stream);
void rsvd_graph_destroy(rsvd_graph_t graph);

/*
 * Draw columns col0 .. col0+cols-1 of the Gaussian family (seed, stream) for
 * rows 0 .. rows-1 into d_out (row-major, leading dimension ld >= cols),
 * dtype RSVD_F64 or RSVD_F32, by the Philox/Box-Muller mapping described at
 * rsvd_desc.seed.  The same numbers rsvd_factor uses for Omega (stream 4).
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_gaussian(uint64_t seed, uint32_t stream_id, int64_t rows, int64_t cols, int64_t col0,
                          int32_t dtype, void* d_out, int64_t ld, void* stream);

/*
 * Raw Philox4x32-10: d_out[4i .. 4i+3] = Philox(d_ctr[4i .. 4i+3], key (k0, k1))
 * for i < count (device uint32 arrays).  Exposed so the generator can be
 * checked against its published known answers.
 * Errors: RSVD_E_ARG, RSVD_E_HIP.
 */
rsvd_status rsvd_philox4x32_10(int64_t count, const uint32_t* d_ctr, uint32_t k0, uint32_t k1,
                               uint32_t* d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H_ */
