/*
 * mc_oracle.c -- plain FP64 CPU oracle of the matrix-condensation
 * log-determinant (arXiv 1811.08057, Eqs. 1-3, Sections 2.2-2.4, Figure 6).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU engine is checked
 * against.  Slow and straightforward on purpose; built with contraction
 * off so every product and difference is rounded on its own.
 */
#include "mc_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads for the row updates of one condensation step (1 = serial).
 * Figure 6 hands the rows of a step to different processes; here they go to
 * OpenMP threads.  Every row's arithmetic is the same with any count, so
 * the results do not depend on it. */
static int g_threads = 1;

int mco_set_threads(int threads)
{
    const int prev = g_threads;
    g_threads = threads < 1 ? 1 : threads;
    return prev;
}

int mco_num_procs(void) { return omp_get_num_procs(); }

/* Compensated (Neumaier) running sum of log|pivot| (Figure 6, step 4.4
 * accumulates log|pivot|; the compensation keeps the sum to ~1 ulp). */
typedef struct {
    double sum, comp;
} neumaier;

static void neumaier_add(neumaier* a, double x)
{
    double t = a->sum + x;
    if (fabs(a->sum) >= fabs(x))
        a->comp += (a->sum - t) + x;
    else
        a->comp += (x - t) + a->sum;
    a->sum = t;
}

/* Sign of a permutation of 0..n-1 by counting its cycles:
 * sgn = (-1)^(n - cycles). */
static int perm_sign(const int32_t* p, int64_t n)
{
    unsigned char* seen = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t cycles = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (seen[i]) continue;
        ++cycles;
        for (int64_t j = i; !seen[j]; j = p[j]) seen[j] = 1;
    }
    free(seen);
    return ((n - cycles) & 1) ? -1 : 1;
}

/* Pivot-column choice in the pivot row (Section 2.2).  row holds the m
 * active slots, colid[j] the original column of slot j.  Ties go to the
 * smallest original column.  Returns the slot, or -1 when no candidate
 * exists (all entries zero). */
static int64_t choose_column(const double* row, const int32_t* colid,
                             int64_t m, int rule)
{
    int64_t best = -1;
    double bestkey = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        double a = fabs(row[j]);
        double key;
        if (rule == MCO_COL_MAXABS) {
            key = a; /* larger is better */
            if (best < 0 || key > bestkey ||
                (key == bestkey && colid[j] < colid[best])) {
                best = j;
                bestkey = key;
            }
        } else if (rule == MCO_COL_FIRST_NONZERO) {
            if (a != 0.0 && (best < 0 || colid[j] < colid[best])) best = j;
        } else { /* MCO_COL_CLOSEST_TO_ONE: smaller | |a| - 1 | is better */
            if (a == 0.0) continue;
            key = fabs(a - 1.0);
            if (best < 0 || key < bestkey ||
                (key == bestkey && colid[j] < colid[best])) {
                best = j;
                bestkey = key;
            }
        }
    }
    if (rule == MCO_COL_MAXABS && best >= 0 && row[best] == 0.0) best = -1;
    return best;
}

/* Row order for the whole run; returns 0 or -1 if the order is invalid. */
static int build_row_order(int64_t n, int policy, const int64_t* given,
                           int64_t n_virt, int64_t* ord)
{
    if (policy == MCO_ROWS_TOP_DOWN) {
        for (int64_t s = 0; s < n; ++s) ord[s] = s;
    } else if (policy == MCO_ROWS_BOTTOM_UP) {
        for (int64_t s = 0; s < n; ++s) ord[s] = n - 1 - s;
    } else if (policy == MCO_ROWS_EXPLICIT) {
        if (!given) return -1;
        unsigned char* used = (unsigned char*)calloc((size_t)n, 1);
        for (int64_t s = 0; s < n; ++s) {
            if (given[s] < 0 || given[s] >= n || used[given[s]]) {
                free(used);
                return -1;
            }
            used[given[s]] = 1;
            ord[s] = given[s];
        }
        free(used);
    } else if (policy == MCO_ROWS_FIG6) {
        /* Figure 6: process p owns rows p*(N/n) .. (p+1)*(N/n)-1 (block
         * distribution, Section 2.1); the loops run "for i over local rows,
         * for p over processes", taking local row i of process p. */
        if (n_virt <= 0 || n % n_virt) return -1;
        int64_t local = n / n_virt, s = 0;
        for (int64_t i = 0; i < local; ++i)
            for (int64_t p = 0; p < n_virt; ++p) ord[s++] = p * local + i;
    } else {
        return -1;
    }
    return 0;
}

/* Relative margin of the chosen pivot over the runner-up in its row:
 * (|p| - max over the other active slots of |a|) / |p|; 1 when no other
 * slot is active.  0 means a tie that only the tie rule decided. */
static double pivot_gap(const double* row, int64_t m, int64_t l)
{
    double second = 0.0;
    for (int64_t j = 0; j < m; ++j)
        if (j != l && fabs(row[j]) > second) second = fabs(row[j]);
    const double a = fabs(row[l]);
    return (a - second) / a;
}

static int slogdet_impl(const double* A, int64_t n, int64_t lda,
                        int row_policy, const int64_t* row_order,
                        int64_t n_virt, int col_rule, int64_t max_steps,
                        mco_result* out, int32_t* piv_row_out,
                        int32_t* piv_col_out, double* piv_val_out,
                        double* piv_gap_out)
{
    if (!out) return -8;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !A) return -1;
    if (col_rule < MCO_COL_MAXABS || col_rule > MCO_COL_CLOSEST_TO_ONE)
        return -7;
    if (n == 0) { /* empty product: det = 1 */
        out->logabsdet = 0.0;
        out->sign = 1.0;
        out->info = MCO_INFO_OK;
        return 0;
    }

    int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (build_row_order(n, row_policy, row_order, n_virt, ord)) {
        free(ord);
        return -4;
    }

    /* Working copy W (row-major, stride n), condensed in place (Section
     * 2.4: the active columns stay in slots 0..m-1 of every live row). */
    double* W = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        memcpy(W + i * n, A + i * lda, sizeof(double) * (size_t)n);
    int32_t* colid = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* piv_row = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* piv_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char* live = (unsigned char*)malloc((size_t)n);
    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        colid[j] = (int32_t)j;
        live[j] = 1;
    }

    neumaier logsum = {0.0, 0.0};
    int64_t negatives = 0;
    int64_t steps_done = 0;
    int status = 0; /* 0 ok, 1 singular, 2 non-finite, 3 partial */
    int64_t bad_step = 0;

    for (int64_t s = 0; s < n; ++s) {
        if (max_steps > 0 && s == max_steps) {
            status = 3;
            break;
        }
        const int64_t m = n - s; /* active size of the current matrix */
        const int64_t k = ord[s];
        double* row = W + k * n;

        /* A non-finite value in the pivot row poisons the result. */
        for (int64_t j = 0; j < m; ++j)
            if (!isfinite(row[j])) status = 2;
        if (status == 2) {
            bad_step = s;
            break;
        }

        /* Figure 6 step 4.1: pivot column l of row k; the pivot keeps its
         * sign (step 4.11 divides by the signed value). */
        const int64_t l = choose_column(row, colid, m, col_rule);
        if (l < 0) { /* pivot row is all zero: det A = 0 */
            status = 1;
            bad_step = s;
            break;
        }
        const double p = row[l];

        /* Step 4.4: accumulate log|pivot|; count negative pivots. */
        piv_row[s] = (int32_t)k;
        piv_col[s] = colid[l];
        if (piv_val_out) piv_val_out[s] = p;
        if (piv_gap_out) piv_gap_out[s] = pivot_gap(row, m, l);
        neumaier_add(&logsum, log(fabs(p)));
        if (p < 0.0) ++negatives;
        live[k] = 0;
        ++steps_done;
        if (m == 1) break; /* the 1 x 1 remainder was the last pivot */

        /* Steps 4.3-4.4: factor the pivot out of row k (Section 2.3), then
         * move the last slot into slot l. */
        for (int64_t j = 0; j < m; ++j) r[j] = row[j] / p;
        r[l] = r[m - 1];

        /* Steps 4.8-4.11 for every live row: stash the multiplier a_il,
         * move the last slot into slot l, then form
         * B*_ij = a_ij - a_il * (a_kj / a_kl)  (Eq. 3 with Eq. 2). */
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && m > 32)
        for (int64_t i = 0; i < n; ++i) {
            if (!live[i]) continue;
            double* wi = W + i * n;
            const double c = wi[l];
            wi[l] = wi[m - 1];
            for (int64_t j = 0; j < m - 1; ++j) {
                const double prod = c * r[j];
                wi[j] = wi[j] - prod;
            }
        }
        colid[l] = colid[m - 1];
    }

    if (status == 1) {
        out->logabsdet = -INFINITY;
        out->sign = 0.0;
        out->info = bad_step + 1;
    } else if (status == 2) {
        out->logabsdet = NAN;
        out->sign = 0.0;
        out->info = MCO_INFO_NONFINITE;
    } else if (status == 3) {
        out->logabsdet = logsum.sum + logsum.comp;
        out->sign = 0.0;
        out->info = MCO_INFO_PARTIAL;
    } else {
        /* det A = sgn(rows) * sgn(cols) * prod(pivots): the steps are LU
         * without further pivoting of A with its rows taken in the order
         * piv_row and its columns in the order piv_col. */
        int sg = (negatives & 1) ? -1 : 1;
        sg *= perm_sign(piv_row, n);
        sg *= perm_sign(piv_col, n);
        double la = logsum.sum + logsum.comp;
        if (!isfinite(la)) {
            out->logabsdet = NAN;
            out->sign = 0.0;
            out->info = MCO_INFO_NONFINITE;
        } else {
            out->logabsdet = la;
            out->sign = (double)sg;
            out->info = MCO_INFO_OK;
        }
    }
    if (piv_row_out)
        memcpy(piv_row_out, piv_row, sizeof(int32_t) * (size_t)steps_done);
    if (piv_col_out)
        memcpy(piv_col_out, piv_col, sizeof(int32_t) * (size_t)steps_done);

    free(ord);
    free(W);
    free(colid);
    free(piv_row);
    free(piv_col);
    free(live);
    free(r);
    return 0;
}

int mco_slogdet(const double* A, int64_t n, int64_t lda, int row_policy,
                const int64_t* row_order, int64_t n_virt, int col_rule,
                mco_result* out, int32_t* piv_row, int32_t* piv_col,
                double* piv_val)
{
    return slogdet_impl(A, n, lda, row_policy, row_order, n_virt, col_rule, 0,
                        out, piv_row, piv_col, piv_val, NULL);
}

int mco_slogdet_gaps(const double* A, int64_t n, int64_t lda, mco_result* out,
                     int32_t* piv_col, double* piv_gap)
{
    return slogdet_impl(A, n, lda, MCO_ROWS_TOP_DOWN, NULL, 0, MCO_COL_MAXABS, 0,
                        out, NULL, piv_col, NULL, piv_gap);
}

int mco_slogdet_steps(const double* A, int64_t n, int64_t lda,
                      int64_t max_steps, mco_result* out)
{
    return slogdet_impl(A, n, lda, MCO_ROWS_TOP_DOWN, NULL, 0, MCO_COL_MAXABS,
                        max_steps, out, NULL, NULL, NULL, NULL);
}

/* 2 x 2 determinant of [[a, b], [c, d]]. */
static double det2(double a, double b, double c, double d)
{
    const double ad = a * d;
    const double bc = b * c;
    return ad - bc;
}

int mco_condense_step(const double* A, int64_t n, int64_t lda, int64_t k,
                      int64_t l, int factored, double* B)
{
    if (n < 2) return -2;
    if (lda < n) return -3;
    if (k < 0 || k >= n) return -4;
    if (l < 0 || l >= n) return -5;
    if (!A || !B) return -1;
#define a(i, j) A[(i) * lda + (j)]
    const double akl = factored ? 1.0 : a(k, l);
    /* a*_kj: row k with the pivot factored out (Eq. 3, Section 2.3). */
#define akj(j) (factored ? a(k, j) / a(k, l) : a(k, j))
    for (int64_t i = 0; i < n - 1; ++i) {
        for (int64_t j = 0; j < n - 1; ++j) {
            double v;
            if (i < k && j < l) /* Eq. 2, first case */
                v = det2(a(i, j), a(i, l), akj(j), akl);
            else if (i < k) /* j >= l */
                v = det2(akl, akj(j + 1), a(i, l), a(i, j + 1));
            else if (j < l) /* i >= k */
                v = det2(akl, akj(j), a(i + 1, l), a(i + 1, j));
            else /* i >= k, j >= l */
                v = det2(akl, akj(j + 1), a(i + 1, l), a(i + 1, j + 1));
            B[i * (n - 1) + j] = v;
        }
    }
#undef akj
#undef a
    return 0;
}

int mco_inverse(const double* A, int64_t n, int64_t lda, double* Ainv,
                int64_t ldi)
{
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (ldi < (n > 1 ? n : 1)) return -5;
    if (n == 0) return 0;
    if (!A || !Ainv) return -1;
    const int64_t w = 2 * n;
    double* M = (double*)malloc(sizeof(double) * (size_t)n * (size_t)w);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            M[i * w + j] = A[i * lda + j];
            M[i * w + n + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    int rc = 0;
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = c;
        for (int64_t i = c + 1; i < n; ++i)
            if (fabs(M[i * w + c]) > fabs(M[piv * w + c])) piv = i;
        if (M[piv * w + c] == 0.0) {
            rc = 1;
            break;
        }
        if (piv != c)
            for (int64_t j = 0; j < w; ++j) {
                double t = M[c * w + j];
                M[c * w + j] = M[piv * w + j];
                M[piv * w + j] = t;
            }
        const double d = M[c * w + c];
        for (int64_t j = 0; j < w; ++j) M[c * w + j] = M[c * w + j] / d;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && n > 32)
        for (int64_t i = 0; i < n; ++i) {
            if (i == c) continue;
            const double f = M[i * w + c];
            if (f == 0.0) continue;
            for (int64_t j = 0; j < w; ++j) {
                const double prod = f * M[c * w + j];
                M[i * w + j] = M[i * w + j] - prod;
            }
        }
    }
    if (rc == 0)
        for (int64_t i = 0; i < n; ++i)
            memcpy(Ainv + i * ldi, M + i * w + n, sizeof(double) * (size_t)n);
    free(M);
    return rc;
}
