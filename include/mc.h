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
 *   - Concurrent calls are safe on different streams with different
 *     workspaces; calls that share a workspace must be stream-ordered.
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

#define MC_INFO_NONFINITE (-1)

/* Library version as major*10000 + minor*100 + patch. */
int mc_version(void);

/* Human-readable text for a status code (static storage). */
const char* mc_status_string(mc_status status);

/*
 * Workspace size in bytes for mc_logdet with the same (n, dtype, update, b).
 * Returns 0 for an invalid combination.
 */
size_t mc_logdet_workspace(int64_t n, int dtype, int update, int64_t b);

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
 * Optional timing of the kernel that dominates a call: the condensation
 * update of the plain path (timed as the whole run of per-step launches).
 * While enabled, each call records a pair of HIP events on its stream
 * around those launches and adds the launches' algorithmic traffic: for
 * the plain path 16 bytes per updated FP64 entry (one read, one write of
 * the live block, Figure 6 step 4.11) and 2 flops per entry.
 *
 * mc_profile_enable(1) resets the counters and starts recording;
 * mc_profile_enable(0) stops.  Host-side, not thread-safe; at most 4096
 * event pairs are kept (later launches are counted but not timed).
 * mc_profile_read synchronises on the recorded events and returns the
 * summed elapsed time (ms), the number of kernel launches covered, and the
 * algorithmic bytes and flops of those launches.  Pointers are host
 * pointers; any may be NULL.
 */
mc_status mc_profile_enable(int on);
mc_status mc_profile_read(double* elapsed_ms, int64_t* launches,
                          double* alg_bytes, double* alg_flops);

#ifdef __cplusplus
}
#endif

#endif /* MC_H */
