/*
 * mc.h -- C ABI of the MI355X (gfx950) matrix-condensation log-determinant
 * engine (method: Dong, Barnett, Dhall, arXiv 1811.08057).
 *
 * The engine computes (sign det A, log|det A|) by repeated condensation
 * (Eqs. 1-3): at each step the pivot row k is the next row from the top,
 * its pivot column l is the column of largest |a_kl| (Section 2.2; ties go
 * to the smallest original column index), the pivot is factored out of
 * row k (Section 2.3), log|a_kl| and its sign are accumulated (Figure 6,
 * step 4.4), and the remaining (N-1) x (N-1) matrix is formed from the 2x2
 * determinants of Eq. 2 in the compact form of Figure 6, step 4.11.
 *
 * Conventions shared by every entry point:
 *   - Matrices are row-major: element (i, j) of A is A[i * lda + j], with
 *     lda >= max(1, n) counted in elements (Section 2.6 assumes row-major
 *     storage).  Because pivots are searched along rows, the pivot sequence
 *     depends on the orientation; the determinant does not.
 *   - Every pointer argument except `out` of the query calls is a DEVICE
 *     pointer on the current HIP device.  `stream` is a hipStream_t (NULL
 *     selects the null stream).  All work is enqueued on `stream`; the call
 *     returns without waiting for it.
 *   - The caller owns and allocates all memory, including the workspace
 *     (size from the matching *_workspace query).  The library allocates no
 *     device memory and keeps no pointer after a call returns.
 *   - Return value (mc_status): MC_OK, or a negative code checked on the
 *     host BEFORE anything is enqueued: -i for an invalid i-th argument
 *     (LAPACK style), or one of the MC_ERR_* codes.  Numerical outcomes are
 *     not errors; they are written asynchronously into the mc_result.
 *   - Results: a singular matrix (an all-zero pivot row at 0-based step s)
 *     gives {logabsdet = -inf, sign = 0, info = s + 1}; a NaN or Inf in a
 *     pivot row gives {NaN, 0, MC_INFO_NONFINITE}; n = 0 gives {0, +1, 0}.
 *   - Concurrency.  Calls on different streams need different workspaces;
 *     calls that share a workspace must be stream-ordered.  Blocked-path
 *     calls (mc_logdet / mc_logdet_pivots with b != 0, mc_logdet_factor and
 *     the calls built on it) run one after another on the GPU per device,
 *     whatever streams they are enqueued on: each waits for an event the
 *     device's previous blocked call recorded after its last kernel,
 *     because a column-split panel (below) needs all of its blocks resident
 *     together on one XCD and two panels at once would contend for them.
 *     Calls enqueued under graph capture are not ordered that way; a
 *     replayed graph must not overlap another blocked call on its device.
 *     A foreign kernel that holds the panel XCD's compute units for more
 *     than a second makes the call end with MC_INFO_ABORTED (its bounded
 *     waits run out) rather than hang.  The plain and batched paths keep
 *     no such state.  Process-wide settings (mc_lookahead_enable,
 *     mc_split_panel_enable) are atomic and read once per call.
 */
#ifndef MC_H
#define MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage type of the input matrix. */
typedef enum { MC_DTYPE_F64 = 0, MC_DTYPE_F32 = 1 } mc_dtype;

/* Arithmetic of the condensation updates.  Pivot search, the sum of
 * log|pivot| (compensated, FP64) and the sign parity are FP64/exact in
 * every mode.
 *   MC_UPDATE_NATIVE  updates in the storage type;
 *   MC_UPDATE_F32     blocked trailing updates on FP32 matrix cores;
 *   MC_UPDATE_BF16X3  blocked trailing updates as three BF16 products
 *                     (hi*hi + hi*lo + lo*hi) with FP32 accumulation. */
typedef enum {
    MC_UPDATE_NATIVE = 0,
    MC_UPDATE_F32 = 1,
    MC_UPDATE_BF16X3 = 2
} mc_update;

typedef struct {
    double logabsdet; /* log|det A|                                   */
    double sign;      /* -1, 0 or +1                                  */
    int64_t info;     /* 0, s+1 (singular at step s), or < 0          */
} mc_result;

typedef int mc_status;

#define MC_OK 0
#define MC_ERR_WORKSPACE (-100)   /* work_bytes below the query's size   */
#define MC_ERR_HIP (-101)         /* a HIP launch or query failed        */
#define MC_ERR_UNSUPPORTED (-102) /* combination not provided            */
#define MC_ERR_TOO_LARGE (-103)   /* mc_logdet_noalloc: the workspace the
                                     call needs exceeds MC_NOALLOC_BYTES  */

#define MC_INFO_NONFINITE (-1)
#define MC_INFO_BADARG (-3) /* batched: this matrix's n / lda / pointer invalid */
#define MC_INFO_ABORTED (-4) /* an internal bounded wait ran out (a bug) */

/* Library version as major*10000 + minor*100 + patch. */
int mc_version(void);

/* Human-readable text for a status code (static storage). */
const char* mc_status_string(mc_status status);

/* Text of the last HIP error seen by a call on this host thread that
 * returned MC_ERR_HIP ("no error" if none). */
const char* mc_last_hip_error(void);

/*
 * Workspace size in bytes for mc_logdet with the same (n, dtype, update, b).
 * Returns 0 for an invalid combination.
 */
size_t mc_logdet_workspace(int64_t n, int dtype, int update, int64_t b);

/*
 * The panel width the blocked path uses for b < 0 (the library default) on
 * an n x n matrix of the given mc_dtype: 32 up to n = 256, 64 up to 1024,
 * 128 above.  n < 0: 0.
 */
int64_t mc_default_panel(int64_t n, int dtype);

/*
 * log|det A| and sign of one n x n matrix.
 *
 * A       device, row-major n x n, row stride lda (elements); read only.
 * n       >= 0.
 * lda     >= max(1, n).
 * dtype   mc_dtype of A.
 * update  mc_update (MC_UPDATE_NATIVE for the plain path).
 * b       panel width.  0 = plain (unblocked) condensation, one step per
 *         pivot with the paper's column slot move (Section 2.4, Figure 6);
 *         FP64 storage only.  1..128 = panel-blocked (delayed-update)
 *         condensation: b steps on a panel of b rows, then one trailing
 *         update of the rows below on the matrix cores (block condensation,
 *         Section 2.5 / Future Work).  < 0 = the library's default width.
 *         Supported: (F64, NATIVE) plain or blocked; (F32, NATIVE | F32 |
 *         BF16X3) blocked.  Others return MC_ERR_UNSUPPORTED.
 * out     device pointer to one mc_result, written on `stream`.
 * work    device workspace of at least mc_logdet_workspace(...) bytes,
 *         256-byte aligned.  Its contents on entry are ignored.
 * stream  hipStream_t.
 */
mc_status mc_logdet(const void* A, int64_t n, int64_t lda, int dtype,
                    int update, int64_t b, mc_result* out, void* work,
                    size_t work_bytes, void* stream);

/*
 * As mc_logdet, and also the pivot sequence: piv_col[s] is the ORIGINAL
 * column index of the pivot chosen at step s (row s of A), s = 0..n-1 --
 * the column of largest |a| in the condensed row s, ties to the smallest
 * original index (Section 2.2; Figure 6 step 4.1).  The sequence is the
 * same on the plain and the blocked paths (the plain path's slot moves of
 * Section 2.4 and the blocked path's position exchanges only change where
 * a column sits, not which original column a step takes).
 *
 * piv_col  device, n int32 (output; n = 0: may be NULL).  Written on
 *          `stream`.  Meaningful when out->info == 0; after a singular or
 *          non-finite result its entries from the failing step on are
 *          unspecified.
 * Other arguments as mc_logdet; argument numbers in error returns count
 * piv_col as argument 7 (out is 8, work 9).
 */
mc_status mc_logdet_pivots(const void* A, int64_t n, int64_t lda, int dtype,
                           int update, int64_t b, int32_t* piv_col,
                           mc_result* out, void* work, size_t work_bytes,
                           void* stream);

/*
 * mc_logdet without a workspace argument, for callers that cannot allocate
 * device memory: code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The library allocates nothing for it either: the
 * workspace is a fixed device array of MC_NOALLOC_BYTES inside the library,
 * one per GPU, held until the process ends.  Calls that need more than that
 * (mc_logdet_workspace(n, dtype, update, b) > MC_NOALLOC_BYTES; n = 2048 fits
 * every path) return MC_ERR_TOO_LARGE before anything is enqueued.
 *
 * Arguments, results and error numbering as mc_logdet (without work and
 * work_bytes).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams, or different host threads without
 * stream ordering) race and must not be made.  The blocked path runs with
 * lookahead off and creates no stream or event (mc_lookahead_enable does not
 * apply); it is not ordered against other blocked calls on the device, which
 * must not overlap it either.  The first call on each device looks the
 * array's device address up (hipGetSymbolAddress); make that first call
 * outside graph capture.
 */
#define MC_NOALLOC_BYTES (40u * 1024u * 1024u)
mc_status mc_logdet_noalloc(const void* A, int64_t n, int64_t lda, int dtype,
                            int update, int64_t b, mc_result* out,
                            void* stream);

/*
 * Pivot-column rules inside the pivot row.  The paper's rule is the column
 * of largest |a_kl| (Section 2.2).  Section 1 describes two earlier rules
 * that the paper argues against (Section 2.2: a tiny pivot can lose digits
 * or overflow the running product): the first non-zero entry of the row
 * (Beliakov) and the non-zero entry whose |a| is closest to 1 (Haque).
 * Ties go to the smallest original column under every rule.
 */
#define MC_PIVOT_MAXABS 0
#define MC_PIVOT_FIRST_NONZERO 1
#define MC_PIVOT_CLOSEST_TO_ONE 2

/*
 * The plain (unblocked) FP64 condensation of mc_logdet with b = 0 under a
 * chosen pivot-column rule (MC_PIVOT_*), for studying the rules' accuracy;
 * MC_PIVOT_MAXABS is exactly mc_logdet_pivots with b = 0.  Under the other
 * two rules a row with no non-zero entry is singular as before; otherwise
 * the step takes the rule's choice however small it is.
 *
 * A        device, row-major n x n FP64, row stride lda; read only.
 * rule     MC_PIVOT_MAXABS, MC_PIVOT_FIRST_NONZERO or MC_PIVOT_CLOSEST_TO_ONE.
 * piv_col  device, n int32 (output), or NULL: the original column of each
 *          step's pivot, as in mc_logdet_pivots.
 * out      device mc_result.
 * work     >= mc_logdet_workspace(n, MC_DTYPE_F64, MC_UPDATE_NATIVE, 0)
 *          bytes, 256-byte aligned.
 * Error returns number the arguments A = 1, n = 2, lda = 3, rule = 4,
 * out = 6, work = 7.
 */
mc_status mc_logdet_rule(const void* A, int64_t n, int64_t lda, int rule,
                         int32_t* piv_col, mc_result* out, void* work,
                         size_t work_bytes, void* stream);

/*
 * Factor call: the blocked condensation of mc_logdet run in place, keeping
 * the factors (the row-k factoring of Section 2.3 with the multipliers of
 * Figure 6 step 4.8 stored where they were eliminated).  On return A holds
 * L\U with A_in[:, perm] = L U: row i keeps its multipliers left of i (L),
 * its pivot at i (diagonal of L) and its factored row right of i (U, unit
 * diagonal implied); perm[s] is the original column of position s.
 *
 * A       device, row-major n x n, row stride lda; overwritten.
 * b       panel width (1..128) or < 0 for the default; b = 0 is rejected.
 * perm    device, n int32 (output).
 * out     device mc_result (as mc_logdet).
 * work    >= mc_logdet_factor_workspace(n, dtype, update, b) bytes.
 * After a singular or non-finite result, A and perm are unspecified.
 */
size_t mc_logdet_factor_workspace(int64_t n, int dtype, int update,
                                  int64_t b);
mc_status mc_logdet_factor(void* A, int64_t n, int64_t lda, int dtype,
                           int update, int64_t b, int32_t* perm,
                           mc_result* out, void* work, size_t work_bytes,
                           void* stream);

/*
 * Backward call: gradA = g * A^{-T} = g * d log|det A| / dA from the output
 * of mc_logdet_factor (LU with row stride ld, perm).  A^{-1} = Q U^{-1}
 * L^{-1}: two blocked triangular substitutions whose off-diagonal updates
 * run on the matrix cores, then a permuted transpose.  (The paper computes
 * only the forward value; the gradient is what the covariance workloads of
 * its Abstract need to fit a model.)
 *
 * LU, ld    device, row-major factors from mc_logdet_factor (read only).
 * perm      device, n int32 from the same call.
 * dtype     mc_dtype of LU and gradA.
 * grad_out  device pointer to one double g (the incoming gradient of
 *           log|det A|), or NULL for g = 1.
 * fwd       device pointer to the factor call's mc_result, or NULL.  When
 *           given and its info != 0 (singular, non-finite or aborted) the
 *           factors are not a valid L U: every entry of gradA is NaN
 *           (checked on the device; no host synchronisation).  When NULL the
 *           factors must come from a call whose result had info == 0.
 * gradA     device, row-major n x n, row stride ldg (output).
 * work      >= mc_logdet_backward_workspace(n, dtype) bytes, 256-aligned.
 */
size_t mc_logdet_backward_workspace(int64_t n, int dtype);
mc_status mc_logdet_backward(const void* LU, int64_t n, int64_t ld,
                             const int32_t* perm, int dtype,
                             const double* grad_out, const mc_result* fwd,
                             void* gradA, int64_t ldg, void* work,
                             size_t work_bytes, void* stream);

/*
 * Backward with the factors recomputed (for callers that did not keep
 * them): factors a copy of A inside `work` exactly as mc_logdet_factor
 * would (same b, update and pivots), then runs mc_logdet_backward on it
 * with the forward result as `fwd`.  A is read only.
 *
 * out    device mc_result of the recomputed forward (optional; NULL: kept
 *        inside the workspace).
 * work   >= mc_logdet_backward_recompute_workspace(n, dtype, update, b)
 *        bytes, 256-aligned: a copy of A, perm, the result, and one region
 *        the factorisation and then the substitutions use.
 * Other arguments as mc_logdet_factor and mc_logdet_backward.
 */
size_t mc_logdet_backward_recompute_workspace(int64_t n, int dtype,
                                              int update, int64_t b);
mc_status mc_logdet_backward_recompute(const void* A, int64_t n, int64_t lda,
                                       int dtype, int update, int64_t b,
                                       const double* grad_out, void* gradA,
                                       int64_t ldg, mc_result* out,
                                       void* work, size_t work_bytes,
                                       void* stream);

/*
 * Batched log-determinants of `batch` independent square matrices of
 * possibly different sizes (e.g. the covariance matrices of a mixture
 * model, Abstract), in one persistent kernel launch preceded by a one-block
 * setup launch; the pair can be captured in a hipGraph.  Each workgroup
 * takes the largest remaining matrix from a queue and condenses it alone
 * with the blocked algorithm (largest-|a| pivot per row, row factoring,
 * trailing updates on the matrix cores).
 *
 * A_array    device array of `batch` device pointers (row-major matrices).
 * n_array    device array of `batch` sizes (int64, 0 <= n_k <= n_max).
 * lda_array  device array of `batch` row strides (int64, >= max(1, n_k)).
 * batch      >= 0.
 * n_max      host value: an upper bound of every n_k; sizes the per-matrix
 *            workspace regions.  A matrix that breaks n_k <= n_max (or has
 *            an invalid lda or a NULL pointer) gets {NaN, 0, MC_INFO_BADARG}
 *            and the others are unaffected.
 * dtype      MC_DTYPE_F64 (update NATIVE) or MC_DTYPE_F32 (update NATIVE,
 *            F32 or BF16X3).
 * b          > 0: this panel width for every matrix (1..128); < 0: the
 *            per-size table (mc_tune_get / mc_autotune_batched); 0 is
 *            rejected (the plain path is mc_logdet with b = 0).
 * out        device array of `batch` mc_result.
 * work       >= mc_logdet_batched_workspace(batch, n_max, dtype, update, b)
 *            bytes, 256-byte aligned; after the call it holds each matrix's
 *            factors in its region (contents otherwise unspecified).
 */
size_t mc_logdet_batched_workspace(int64_t batch, int64_t n_max, int dtype,
                                   int update, int64_t b);
mc_status mc_logdet_batched(const void* const* A_array, const int64_t* n_array,
                            const int64_t* lda_array, int64_t batch,
                            int64_t n_max, int dtype, int update, int64_t b,
                            mc_result* out, void* work, size_t work_bytes,
                            void* stream);

/*
 * Batched factor call: mc_logdet_batched with each matrix condensed in
 * place and its factors kept, exactly as mc_logdet_factor leaves them
 * (A_k,in[:, perm_k] = L_k U_k, L\U in A_k; Section 2.3 and Figure 6 step
 * 4.8), so that mc_logdet_batched_backward (or mc_logdet_backward per
 * matrix) can use them.  One persistent launch (plus a one-block setup
 * launch), graph-capturable.
 *
 * A_array     device array of `batch` device pointers; overwritten.
 * perm_array  device array of `batch` device pointers to n_k int32 each
 *             (output; n_k = 0: may be NULL).
 * Other arguments as mc_logdet_batched (error numbering: A_array 1,
 * n_array 2, lda_array 3, perm_array 4, batch 5, n_max 6, dtype 7,
 * update 8, b 9, out 10, work 11).  The workspace holds no copy of the
 * matrices (it is smaller than mc_logdet_batched's).  After a singular or
 * non-finite result, that matrix and its perm are unspecified.
 */
size_t mc_logdet_batched_factor_workspace(int64_t batch, int64_t n_max,
                                          int dtype, int update, int64_t b);
mc_status mc_logdet_batched_factor(void* const* A_array, const int64_t* n_array,
                                   const int64_t* lda_array,
                                   int32_t* const* perm_array, int64_t batch,
                                   int64_t n_max, int dtype, int update,
                                   int64_t b, mc_result* out, void* work,
                                   size_t work_bytes, void* stream);

/*
 * Batched backward call: G_k = g_k * A_k^{-T} for every member, from the
 * factors of mc_logdet_factor or mc_logdet_batched_factor, in one
 * persistent launch (plus a one-block setup launch; graph-capturable).  The
 * work is split into (matrix, 64-column block) items taken largest matrix
 * first; each item runs the two triangular substitutions of its columns of
 * A^{-1} = Q U^{-1} L^{-1} with the block updates on the matrix cores.
 *
 * LU_array, perm_array  device arrays of `batch` device pointers: factors
 *             (row stride ld_array[k]) and perms; read only.
 * n_array, ld_array     device arrays of `batch` int64.
 * n_max       host value, 0 <= n_max <= 16384: an upper bound of every n_k
 *             (members with n_k outside [0, n_max] are skipped, G_k left
 *             untouched).
 * dtype       mc_dtype of the factors and gradients.
 * grad_out    device array of `batch` doubles (g_k), or NULL for g_k = 1.
 * fwd         device array of the `batch` factor results, or NULL; a member
 *             whose info != 0 gets an all-NaN G_k.
 * G_array     device array of `batch` device pointers (output, n_k x n_k,
 *             row stride ldg_array[k]); must not overlap the factors.
 *             G_k's rows also serve as the item's working storage.
 * work        >= mc_logdet_batched_backward_workspace(batch, n_max, dtype)
 *             bytes, 256-byte aligned (the item queue).
 * Error numbering: LU_array 1, n_array 2, ld_array 3, perm_array 4,
 * batch 5, n_max 6, dtype 7, G_array 10, ldg_array 11, work 12.
 */
size_t mc_logdet_batched_backward_workspace(int64_t batch, int64_t n_max,
                                            int dtype);
mc_status mc_logdet_batched_backward(const void* const* LU_array,
                                     const int64_t* n_array,
                                     const int64_t* ld_array,
                                     const int32_t* const* perm_array,
                                     int64_t batch, int64_t n_max, int dtype,
                                     const double* grad_out,
                                     const mc_result* fwd,
                                     void* const* G_array,
                                     const int64_t* ldg_array, void* work,
                                     size_t work_bytes, void* stream);

/*
 * Log-likelihood of a Gaussian mixture (the use of the log-determinant the
 * paper's Abstract names: the log-likelihood of model mixtures), from the
 * factors of its covariances:
 *   loglik[i] = log sum_k exp( log_weights[k]
 *                 - (d log(2 pi) + log|Sigma_k| + q_k(x_i)) / 2 ),
 *   q_k(x) = (x - mu_k)^T Sigma_k^{-1} (x - mu_k),
 * with log|Sigma_k| the factor call's result and q_k by two blocked
 * triangular substitutions per block of 64 points on the kept factors
 * (Sigma_k^{-1} = Q U^{-1} L^{-1}), block updates on the matrix cores; the
 * sum over components in FP64, shifted by its largest term.
 *
 * X          device, m x d row-major points (row stride ldx >= d).
 * means      device, k x d row-major (row stride ldmu >= d).
 * log_weights device, k doubles: log pi_k.
 * LU_array, ld_array, perm_array  device arrays of k entries: each
 *            component's factors as mc_logdet_factor or
 *            mc_logdet_batched_factor leave them (d x d).
 * fwd        device, the k factor results; a component whose info != 0 or
 *            whose sign is not +1 (not a covariance) makes every loglik NaN.
 * dtype      mc_dtype of X, means and the factors (the terms accumulate in
 *            that type, the sum over components in FP64).
 * loglik     device, m doubles (output).
 * total      device, one double: sum_i loglik[i] (output), or NULL.
 * work       >= mc_gmm_loglik_workspace(m, d, k, dtype) bytes, 256-aligned.
 * d <= 16384.  Error numbering follows the argument order (X = 1 ...
 * work = 16).  Graph-capturable (the queue is reset by a kernel).
 */
size_t mc_gmm_loglik_workspace(int64_t m, int64_t d, int64_t k, int dtype);
mc_status mc_gmm_loglik(const void* X, int64_t m, int64_t d, int64_t ldx,
                        const void* means, int64_t ldmu, int64_t k,
                        const double* log_weights, const void* const* LU_array,
                        const int64_t* ld_array,
                        const int32_t* const* perm_array, const mc_result* fwd,
                        int dtype, double* loglik, double* total, void* work,
                        size_t work_bytes, void* stream);

/*
 * The batched path's tuning table: for size buckets n <= 64, 128, 256, 512,
 * 1024 and larger, a panel width b_k (1..128) and a trailing-update tile
 * edge tile_k (32 or 64).  One table per (dtype, update), process-wide,
 * host-side, not thread-safe.  mc_tune_get/mc_tune_set copy 6 entries of
 * each array (host pointers).
 *
 * mc_autotune_batched times candidate (b, tile) pairs per bucket on
 * synthetic diagonally dominant matrices generated on the device in `work`
 * (at least mc_autotune_workspace(dtype) bytes), keeps the fastest per
 * bucket in the table, and synchronises `stream`.  Buckets above
 * n_max_tune are left unchanged.
 */
mc_status mc_tune_get(int dtype, int update, int64_t* b, int* tile);
mc_status mc_tune_set(int dtype, int update, const int64_t* b,
                      const int* tile);
size_t mc_autotune_workspace(int dtype, int64_t n_max_tune);
mc_status mc_autotune_batched(int dtype, int update, int64_t n_max_tune,
                              void* work, size_t work_bytes, void* stream);

/*
 * Blocked path scheduling (lookahead).  On (the default), a panel's
 * trailing update is split when the next panel is a column-split panel
 * (see mc_split_panel_enable) and the device exposes all eight of its XCDs:
 * the rows of the next panel are updated on the caller's stream, the
 * remaining rows on a second stream the library owns (one per device,
 * default priority), where that update runs beside the next panel's
 * factorisation.  The panel then runs on XCD 0 and the update on the other
 * seven.  The caller's stream waits for the update (an event) before the
 * next triangular solve and before the call's last kernel, so from the
 * caller's side the call is still ordered on its stream (and can be
 * captured into a graph).  Other panels, and every panel with lookahead
 * off, run each kernel on the caller's stream.  Both schedules give the
 * same pivots and factors.  Returns the previous setting (1 on, 0 off).
 * Process-wide and atomic; a call reads it once, when it starts enqueuing
 * (calls that enqueue blocked work are serialised on a lock while they
 * do).  (Measured on MI355X at N = 8000, FP64: 24.7 ms on,
 * 33.2 ms off.)
 */
int mc_lookahead_enable(int on);

/*
 * Blocked path: choice of panel kernel for panels whose active width
 * (n minus the panel's first step) is at most 8192 (Sections 2.2-2.4 on the
 * panel's rows).  On (the default): one kernel per panel on the compute
 * units of one XCD, each holding a slice of the panel's columns for all of
 * its rows; a step exchanges only a pivot candidate and one column of
 * multipliers per unit.  Off: the row-per-block panel kernels.  Both give
 * the same pivots and the same factors up to rounding order.  Off also
 * turns lookahead's second stream off (it only runs beside column-split
 * panels).  Returns the previous setting (1 on, 0 off).  Process-wide and
 * atomic; a call reads it once, when it starts enqueuing, and keeps it for
 * all of its panels.
 */
int mc_split_panel_enable(int on);

/*
 * Batched launches (mc_logdet_batched, mc_logdet_batched_factor) beside a
 * blocked-path call.  On: the persistent kernel's workgroups that land on
 * XCD 0 leave before taking a matrix, so the launch can run on one stream
 * while blocked-path calls run on another (their column-split panels run on
 * XCD 0 beside their trailing updates): the many small members of a batch
 * on the other XCDs while its largest members go through the blocked path.
 * Off (the default): the launch uses every XCD.  Results are the same
 * either way.  Returns the previous setting (1 on, 0 off).  Process-wide
 * and atomic; a call reads it once, when it enqueues.
 */
int mc_batched_spare_xcd0(int on);

/*
 * Optional timing of the kernels that dominate a call, in two kinds:
 *
 * MC_PROF_UPDATE  the condensation update.  Plain path: the whole run of
 *                 per-step launches, 16 algorithmic bytes (one read, one
 *                 write of the live block, Figure 6 step 4.11) and 2 flops
 *                 per updated FP64 entry.  Blocked path: each trailing
 *                 update launch (Section 2.5's block form), 2 m N b flops
 *                 and sizeof(T) (2 m N + m b + b N) bytes for an m x N
 *                 update of panel width b.
 * MC_PROF_PANEL   the blocked path's panel-chain kernel (the b condensation
 *                 steps of one panel, one launch per panel): the panel's
 *                 rows read once and written once, 2 b w sizeof(T) bytes for
 *                 w active columns, and about 2 b^2 w / 2 flops.
 *
 * While enabled, each such launch is bracketed by a pair of HIP events on
 * the stream it runs on.  mc_profile_enable(1) resets the counters and
 * starts recording; mc_profile_enable(0) stops.  Host-side, not
 * thread-safe; at most 4096 event pairs are kept (later launches are
 * counted but not timed).  mc_profile_read synchronises on the recorded
 * events of one kind and returns their summed elapsed time (ms), the number
 * of kernel launches covered, and the algorithmic bytes and flops of those
 * launches.  Pointers are host pointers; any may be NULL.  kind other than
 * the two: -1.
 */
#define MC_PROF_UPDATE 0
#define MC_PROF_PANEL 1
mc_status mc_profile_enable(int on);
mc_status mc_profile_read(int kind, double* elapsed_ms, int64_t* launches,
                          double* alg_bytes, double* alg_flops);

#ifdef __cplusplus
}
#endif

#endif /* MC_H */
