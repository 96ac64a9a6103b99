// mc_plain.hip -- the plain (unblocked) condensation path on gfx950.
//
// One kernel launch per condensation step (Figure 6 with one process):
//   step s, active size m = n - s, pivot row s, pivot slot l, pivot p:
//     c_i   = W[i][l]                 stash the multiplier   (step 4.8)
//     W[i][l] <- W[i][m-1]            slot move              (step 4.9, Sec. 2.4)
//     W[i][j] <- W[i][j] - c_i * r_j  for j < m-1            (step 4.11, Eq. 2/3)
//   with r = (row s) / p, r_l <- r_{m-1}                    (steps 4.3-4.4)
// Rows below the pivot row are live; the active columns stay in slots
// 0..m-1 of every row (the paper's column exchange keeps them contiguous).
//
// Lookahead: block 0 of step s owns row s+1, the next pivot row.  When it
// has updated that row it finds the next pivot (wavefront-shuffle argmax),
// records it, and writes r for step s+1 = row / pivot into the other half
// of a ping-pong buffer.  No host round trip happens between steps.
//
// Every other block owns `rows_per_block` consecutive rows and streams them
// column by column: each thread keeps r_j in a register for all its rows, so
// r is read once per block while W is read and written once per step.  That
// is the roofline of this path: 16 bytes of HBM (or cache) traffic per
// 2 flops.
#include "mc_device.h"
#include "mc_internal.h"

#include <algorithm>

namespace mc {

constexpr int kPlainThreads = 256;

template <int RULE>
__global__ void __launch_bounds__(kPlainThreads)
plain_init(const double* __restrict__ A, int64_t n, PlainWork w)
{
    __shared__ PivotKey sh[kPlainThreads / kWave];
    __shared__ int shflag;
    __shared__ double shp;
    const int tid = threadIdx.x;
    PivotKey k = no_candidate();
    bool bad = false;
    for (int64_t j = tid; j < n; j += kPlainThreads) {
        w.colid[j] = (int)j;
        if (!offer<RULE>(k, A[j], (int)j, (int)j)) bad = true;
    }
    k = block_argmax<kPlainThreads>(k, bad, sh, &shflag);
    if (tid == 0) {
        int st = kStatusOk;
        if (bad)
            st = kStatusNonfinite;
        else if (k.slot < 0 || k.value == 0.0)
            st = kStatusSingular;
        w.state->status = st;
        w.state->bad_step = 0;
        w.piv_val[0] = k.value;
        w.piv_slot[0] = k.slot;
        if (w.piv_col) w.piv_col[0] = k.colid;
        shp = k.value;
        shflag = st;
    }
    __syncthreads();
    if (shflag != kStatusOk) return;
    const double p = shp;
    for (int64_t j = tid; j < n; j += kPlainThreads) w.r[0][j] = A[j] / p;
}

// src/lds: the matrix rows for this step (the caller's A at step 0, the
// workspace afterwards).  dst is always the workspace.
template <int RULE>
__global__ void __launch_bounds__(kPlainThreads)
plain_step(const double* src, int64_t lds, int64_t n, int64_t s,
           int rows_per_block, PlainWork w)
{
    __shared__ double cs[kMaxRowsPerBlock];
    __shared__ PivotKey sh[kPlainThreads / kWave];
    __shared__ int shflag;
    __shared__ double shp;

    if (w.state->status != kStatusOk) return;
    const int tid = threadIdx.x;
    const int64_t m = n - s;     // active size at this step
    const int64_t wn = m - 1;    // active size after it
    const int l = w.piv_slot[s]; // pivot slot in row s
    const double* __restrict__ rc = w.r[s & 1];
    double* __restrict__ W = w.W;
    const int64_t ldw = w.ldw;

    if (blockIdx.x == 0) {
        // ---- the next pivot row: update, argmax, publish ----
        const int64_t i = s + 1;
        if (tid == 0) {
            cs[0] = src[i * lds + l];
            w.colid[l] = w.colid[m - 1];
        }
        __syncthreads();
        const double c = cs[0];
        PivotKey k = no_candidate();
        bool bad = false;
        for (int64_t j = tid; j < wn; j += kPlainThreads) {
            const int64_t jj = (j == l) ? m - 1 : j;
            const double y = fma(-c, rc[jj], src[i * lds + jj]);
            W[i * ldw + j] = y;
            if (!offer<RULE>(k, y, w.colid[j], (int)j)) bad = true;
        }
        k = block_argmax<kPlainThreads>(k, bad, sh, &shflag);
        if (tid == 0) {
            int st = kStatusOk;
            if (bad)
                st = kStatusNonfinite;
            else if (k.slot < 0 || k.value == 0.0)
                st = kStatusSingular;
            w.piv_val[s + 1] = k.value;
            w.piv_slot[s + 1] = k.slot;
            if (w.piv_col) w.piv_col[s + 1] = k.colid;
            if (st != kStatusOk) {
                w.state->bad_step = (int)(s + 1);
                w.state->status = st;
            }
            shp = k.value;
            shflag = st;
        }
        __syncthreads();
        if (shflag != kStatusOk || wn <= 1) return;
        const double p = shp;
        double* __restrict__ rn = w.r[(s + 1) & 1];
        // each thread divides the entries it wrote itself
        for (int64_t j = tid; j < wn; j += kPlainThreads)
            rn[j] = W[i * ldw + j] / p;
        return;
    }

    // ---- bulk rows ----
    const int64_t row0 = s + 2 + (int64_t)(blockIdx.x - 1) * rows_per_block;
    if (row0 >= n) return;
    const int nr = (int)min((int64_t)rows_per_block, n - row0);
    if (tid < nr) cs[tid] = src[(row0 + tid) * lds + l];
    __syncthreads(); // every multiplier read before any slot is overwritten
    for (int64_t j = tid; j < wn; j += kPlainThreads) {
        const int64_t jj = (j == l) ? m - 1 : j;
        const double rj = rc[jj];
        for (int t = 0; t < nr; ++t) {
            const int64_t i = row0 + t;
            W[i * ldw + j] = fma(-cs[t], rj, src[i * lds + jj]);
        }
    }
}

// Sum log|p_s| (compensated), count negative pivots and slot exchanges, and
// write the result.  Sign: det A = sgn(sigma) * prod p_s, where sigma maps a
// step to the original column it eliminated.  With the slot move, sigma
// composed with the reversal of 0..n-1 is a product of one transposition
// per step whose pivot slot was not the last one, so
//   sgn(sigma) = (-1)^(exchanges) * (-1)^(n(n-1)/2).
__global__ void __launch_bounds__(kPlainThreads)
plain_finalize(int64_t n, PlainWork w, mc_result* out)
{
    __shared__ double ssum[kPlainThreads], scomp[kPlainThreads];
    __shared__ int sneg[kPlainThreads];
    const int tid = threadIdx.x;
    const int st = w.state->status;
    if (st == kStatusSingular) {
        if (tid == 0) {
            out->logabsdet = -INFINITY;
            out->sign = 0.0;
            out->info = (int64_t)w.state->bad_step + 1;
        }
        return;
    }
    if (st == kStatusNonfinite) {
        if (tid == 0) {
            out->logabsdet = NAN;
            out->sign = 0.0;
            out->info = MC_INFO_NONFINITE;
        }
        return;
    }
    Compensated acc{0.0, 0.0};
    int parity = 0;
    for (int64_t s = tid; s < n; s += kPlainThreads) {
        const double p = w.piv_val[s];
        comp_add(acc, log(fabs(p)));
        parity += (p < 0.0) ? 1 : 0;
        parity += (w.piv_slot[s] != (int)(n - 1 - s)) ? 1 : 0;
    }
    ssum[tid] = acc.sum;
    scomp[tid] = acc.comp;
    sneg[tid] = parity & 1;
    __syncthreads();
    if (tid == 0) {
        Compensated tot{0.0, 0.0};
        int par = 0;
        for (int t = 0; t < kPlainThreads; ++t) {
            comp_merge(tot, Compensated{ssum[t], scomp[t]});
            par ^= sneg[t];
        }
        par ^= (int)(((n * (n - 1)) / 2) & 1);
        const double la = tot.sum + tot.comp;
        if (!isfinite(la)) {
            out->logabsdet = NAN;
            out->sign = 0.0;
            out->info = MC_INFO_NONFINITE;
        } else {
            out->logabsdet = la;
            out->sign = par ? -1.0 : 1.0;
            out->info = 0;
        }
    }
}

// ---------------------------------------------------------------- launcher

// The per-step launches (plain_init first when `init`).
template <int RULE>
static void plain_steps(const double* A, int64_t n, int64_t lda, PlainWork w,
                        hipStream_t stream, bool init)
{
    if (init) {
        hipLaunchKernelGGL(plain_init<RULE>, dim3(1), dim3(kPlainThreads), 0,
                           stream, A, n, w);
        return;
    }
    for (int64_t s = 0; s + 1 < n; ++s) {
        const int64_t m = n - s;
        const int64_t bulk_rows = m - 2; // rows s+2 .. n-1
        int rpb = 1;
        if (bulk_rows > kPlainTargetBlocks)
            rpb = (int)std::min<int64_t>(kMaxRowsPerBlock,
                                    (bulk_rows + kPlainTargetBlocks - 1) /
                                        kPlainTargetBlocks);
        const int64_t blocks = 1 + (bulk_rows + rpb - 1) / rpb;
        const double* src = (s == 0) ? A : w.W;
        const int64_t lds = (s == 0) ? lda : w.ldw;
        hipLaunchKernelGGL(plain_step<RULE>, dim3((unsigned)blocks),
                           dim3(kPlainThreads), 0, stream, src, lds, n, s, rpb,
                           w);
    }
}

static void plain_dispatch(const double* A, int64_t n, int64_t lda, PlainWork w,
                           hipStream_t stream, int rule, bool init)
{
    if (rule == kRuleFirstNonzero)
        plain_steps<kRuleFirstNonzero>(A, n, lda, w, stream, init);
    else if (rule == kRuleClosestToOne)
        plain_steps<kRuleClosestToOne>(A, n, lda, w, stream, init);
    else
        plain_steps<kRuleMaxAbs>(A, n, lda, w, stream, init);
}

hipError_t launch_plain_f64(const double* A, int64_t n, int64_t lda,
                            PlainWork w, mc_result* out, hipStream_t stream,
                            int rule)
{
    plain_dispatch(A, n, lda, w, stream, rule, true);
    const ProfMark pm = prof_begin(stream);
    plain_dispatch(A, n, lda, w, stream, rule, false);
    // live entries updated over all steps: sum of (m-1)^2, m = n .. 2
    const double nn = (double)(n - 1);
    const double entries = nn * (nn + 1.0) * (2.0 * nn + 1.0) / 6.0;
    prof_end(stream, pm, n - 1, 16.0 * entries, 2.0 * entries);
    hipLaunchKernelGGL(plain_finalize, dim3(1), dim3(kPlainThreads), 0, stream,
                       n, w, out);
    return hipGetLastError();
}

} // namespace mc
