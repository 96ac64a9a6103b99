/*
 * mc_oracle.h -- plain FP64 CPU oracle for the matrix-condensation
 * log-determinant (Dong, Barnett, Dhall, "Parallel Matrix Condensation for
 * Calculating Log-Determinant of Large Matrix", arXiv 1811.08057).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU engine.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or constant with the GPU engine.
 *
 * Storage is row-major with a row stride (lda) in elements, as the paper's
 * implementation assumes (Section 2.6).
 */
#ifndef MC_ORACLE_H
#define MC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Which live row is the pivot row k at each step.  Eq. 2 holds for any k
 * (Section 1, Section 2.1). */
enum {
    MCO_ROWS_TOP_DOWN = 0,  /* k = first live row (the usual order)          */
    MCO_ROWS_BOTTOM_UP = 1, /* k = last live row                             */
    MCO_ROWS_EXPLICIT = 2,  /* k = row_order[s], a permutation of 0..n-1     */
    MCO_ROWS_FIG6 = 3       /* Figure 6 loop order over n_virt row blocks     */
};

/* Pivot-column rule inside the pivot row (Section 1, Section 2.2). */
enum {
    MCO_COL_MAXABS = 0,        /* the paper's rule: largest |a_kl|           */
    MCO_COL_FIRST_NONZERO = 1, /* Beliakov: smallest column with a_kl != 0   */
    MCO_COL_CLOSEST_TO_ONE = 2 /* Haque: non-zero |a_kl| closest to 1        */
};

/* info codes */
#define MCO_INFO_OK 0
#define MCO_INFO_NONFINITE (-1) /* a pivot row held NaN or Inf            */
#define MCO_INFO_PARTIAL (-2)   /* stopped early by a step limit          */

typedef struct {
    double logabsdet; /* log|det A|; -inf when singular, NaN when non-finite */
    double sign;      /* -1, 0 or +1                                         */
    int64_t info;     /* 0, s+1 for a zero pivot row at step s, or < 0       */
} mco_result;

/*
 * Log-determinant by repeated condensation (Eq. 2/3 with row factoring,
 * Section 2.3; column slot move, Section 2.4; Figure 6 with one process).
 *
 * A        n x n row-major input, row stride lda >= max(1, n); not modified.
 * row_order  used with MCO_ROWS_EXPLICIT (a permutation of 0..n-1), else NULL.
 * n_virt   number of row blocks for MCO_ROWS_FIG6 (must divide n).
 * piv_row, piv_col  optional outputs (n entries each): the pivot row and the
 *          original column picked at each step.  piv_val: the pivots.
 * Returns 0, or a negative value for an invalid argument.
 */
int mco_slogdet(const double* A, int64_t n, int64_t lda, int row_policy,
                const int64_t* row_order, int64_t n_virt, int col_rule,
                mco_result* out, int32_t* piv_row, int32_t* piv_col,
                double* piv_val);

/* As mco_slogdet with top-down rows and the max-|a| rule; piv_gap[s]
 * (optional, n entries) receives the relative margin of step s's pivot over
 * the runner-up in its row, (|p| - |a_second|) / |p| (1 when the row has one
 * active slot, 0 for a tie decided by the tie rule).  A test that compares
 * another implementation's pivot sequence with this one's can use it to see
 * whether rounding alone could change a choice. */
int mco_slogdet_gaps(const double* A, int64_t n, int64_t lda, mco_result* out,
                     int32_t* piv_col, double* piv_gap);

/* Threads for the row updates of each step (OpenMP; default 1).  Results
 * do not depend on the count.  Returns the previous setting. */
int mco_set_threads(int threads);

/* Processors OpenMP sees on this host. */
int mco_num_procs(void);

/* As mco_slogdet (top-down rows, max-|a| rule) but stops after max_steps
 * condensation steps; used only to time a bounded sample.  info is
 * MCO_INFO_PARTIAL when the limit was reached. */
int mco_slogdet_steps(const double* A, int64_t n, int64_t lda,
                      int64_t max_steps, mco_result* out);

/*
 * One condensation step, Eq. 2 (factored = 0) or Eq. 3 with the pivot
 * factored out of row k (factored = 1), with 0-based pivot (k, l).
 * B receives the (n-1) x (n-1) result, row-major with stride n-1, in the
 * natural order of Eq. 2 (row k and column l removed).
 */
int mco_condense_step(const double* A, int64_t n, int64_t lda, int64_t k,
                      int64_t l, int factored, double* B);

/*
 * Explicit inverse by Gauss-Jordan elimination on [A | I] with partial
 * pivoting (largest |entry| in the pivot column).  Written separately from
 * the condensation.  Ainv is n x n row-major with stride ldi.
 * Returns 0, 1 if A is singular, or < 0 for an invalid argument.
 */
int mco_inverse(const double* A, int64_t n, int64_t lda, double* Ainv,
                int64_t ldi);

#ifdef __cplusplus
}
#endif

#endif /* MC_ORACLE_H */
