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
  RSVD_E_UNSUPPORTED = -5,  /* valid but not built (e.g. a dtype combination)                  */
  RSVD_E_BREAKDOWN = -6     /* Cholesky of a Gram matrix broke down even after the shifted retry */
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

/*
 * Problem description.
 *   m, n        shape of A (1 <= k+p <= min(m, n)).
 *   k, p        target rank and oversampling; l = k + p columns are sketched
 *               (Section 4; p = 10 is the paper's usual choice).
 *   q           number of power steps of Figure 5 (q >= 0).
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
 *   flags       RSVD_RETURN_RANK_L | RSVD_TIMING.
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
  int32_t orth_retries;    /* Gram Cholesky breakdowns recovered by a shifted retry  */
  int32_t status;          /* same value as the return code                          */
  double err_bound;        /* certificate value (absolute); 0 when eps == 0           */
  double sigma1;           /* D(1)                                                    */
  float stage_ms[8];       /* with RSVD_TIMING: sketch, power, project, small SVD,
                              lift, certificate, fallback, total                     */
  float nn_ms, tn_ms;      /* with RSVD_TIMING: summed durations of the products A*X
                              and A^T*X (HIP events around each launch)              */
  int32_t nn_launches, tn_launches;
  int32_t jacobi_sweeps;   /* sweeps of the small SVD                                 */
  int32_t dropped_cols;    /* numerically dependent columns met by CholeskyQR          */
  double frob_residual;    /* after a fallback: sqrt(||A||_F^2 - ||B||_F^2) (Section 12.4
                              downdating) of the grown basis; -1 otherwise            */
} rsvd_info;

typedef struct rsvd_plan_s* rsvd_plan_t;

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
 * Errors: RSVD_E_ARG (nothing enqueued), RSVD_E_HIP, RSVD_E_NONFINITE,
 * RSVD_E_BREAKDOWN; RSVD_NOT_CERTIFIED (> 0) when eps is missed at max_rank.
 * Reported only when h_info != NULL or eps > 0: device-side conditions
 * (non-finite values, Cholesky breakdown) need a synchronisation to be seen.
 */
rsvd_status rsvd_factor(rsvd_plan_t plan, const void* d_A, int64_t lda, const double* d_Omega,
                        void* d_U, int64_t ldu, double* d_S, void* d_V, int64_t ldv,
                        rsvd_info* h_info);

/* Release a plan (host memory and events only; the workspace stays the
 * caller's). NULL is ignored. */
void rsvd_destroy(rsvd_plan_t plan);

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
 * (0 = two per compute unit).  Blocks are taken largest first from an atomic
 * queue.  Fully asynchronous; no host synchronisation; capturable.
 * Workspace: rsvd_batched_workspace_size(nblk, n_workgroups).
 * Errors: RSVD_E_ARG, RSVD_E_WORKSPACE, RSVD_E_HIP.
 */
rsvd_status rsvd_batched_workspace_size(int32_t nblk, int32_t n_workgroups, size_t* h_bytes);
rsvd_status rsvd_batched(int32_t nblk, const int32_t* d_m, const int32_t* d_n, const float* const* d_A,
                         const int32_t* d_lda, double eps, int32_t rank_cap, uint64_t seed, float* d_U, double* d_S,
                         float* d_V, const int64_t* d_offU, const int64_t* d_offV, int32_t* d_rank,
                         int32_t* d_status, int32_t n_workgroups, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Capture one rsvd_batched call (same arguments) on `stream` (not the NULL
 * stream) into a HIP graph and instantiate it; rsvd_graph_launch replays it
 * on any stream (the buffers named at capture are reused).  The sequence
 * contains kernels only (no memset nodes).
 * Errors: RSVD_E_ARG, RSVD_E_WORKSPACE, RSVD_E_HIP.
 */
typedef struct rsvd_graph_s* rsvd_graph_t;
rsvd_status rsvd_batched_graph_create(int32_t nblk, const int32_t* d_m, const int32_t* d_n,
                                      const float* const* d_A, const int32_t* d_lda, double eps, int32_t rank_cap,
                                      uint64_t seed, float* d_U, double* d_S, float* d_V, const int64_t* d_offU,
                                      const int64_t* d_offV, int32_t* d_rank, int32_t* d_status,
                                      int32_t n_workgroups, void* d_ws, size_t ws_bytes, void* stream,
                                      rsvd_graph_t* h_out);
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
