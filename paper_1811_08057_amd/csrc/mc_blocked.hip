// mc_blocked.hip -- the panel-blocked (delayed-update) condensation path.
//
// The paper leaves block condensation to future work (Section 2.5, Future
// Work).  With rows taken top to bottom, b consecutive condensation steps
// on rows s0..s0+b-1 (the panel) are b steps of Eq. 2/3 restricted to the
// panel, and their combined effect on every row below is
//     L21 = A21 * U11^{-1}          (the rows' multipliers, a triangular solve)
//     A22 <- A22 - L21 * U12        (one rank-b update: a GEMM on MFMA)
// where U = the factored pivot rows (Figure 6 steps 4.3-4.4) and A21 holds
// the rows' entries in the b pivot columns.  The pivot rule (largest |a|,
// Section 2.2) and the row factoring (Section 2.3) are unchanged; only the
// order in which the products of step 4.11 are summed differs.
//
// Column exchanges: the paper moves the last active column into the pivot
// slot (Section 2.4).  Here the pivot column is exchanged with the column at
// the step's own position instead (the exchange keeps the active block
// [s, n) contiguous just the same), so that after the panel the b pivot
// columns sit at positions s0..s0+b-1 and the factors stay in place: row s
// holds its multipliers left of s, its pivot at s and its factored row
// right of s.  The exchanges are applied to the panel rows as they happen
// and folded into the loads of the rows below (no separate swap pass).
//
// Per panel (b steps, one kernel each, plus four kernels):
//   blk_head   argmax + factoring of the panel's first row
//   blk_step   one step on the panel rows; the block owning the next panel
//              row also finds and factors the next pivot (lookahead)
//   blk_perm   source position of every column the exchanges moved
//   blk_trsm   L21 = gather(A21) * U11^{-1}
//   gemm       A22 <- gather(A22) - L21 * U12    (mc_gemm.hip)
#include <algorithm>

#include "mc_device.h"
#include "mc_gemm.h"
#include "mc_internal.h"

namespace mc {

constexpr int kBlkThreads = 256;
constexpr int kTrsmRows = 64; // rows per solve block (4 lanes per row)

template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_init(const T* __restrict__ A, int64_t lda, int64_t n, BlkWork<T> w)
{
    const int64_t i = blockIdx.x;
    for (int64_t j = threadIdx.x; j < n; j += kBlkThreads)
        w.W[i * w.ldw + j] = A[i * lda + j];
    if (i == 0) {
        for (int64_t j = threadIdx.x; j < n; j += kBlkThreads) {
            w.perm[j] = (int)j;
            w.colsrc[j] = (int)j;
        }
        for (int t = threadIdx.x; t < kMaxPanel; t += kBlkThreads)
            w.moved[t] = -1;
        if (threadIdx.x == 0) {
            w.state->status = kStatusOk;
            w.state->bad_step = 0;
        }
    }
}

// Record the pivot of step s chosen in row s and write the row in factored
// form: position s <- p, position l <- (old value at s) / p, every other
// position j > s <- value / p.  `vs` is the row's value at s before this.
// Called by all threads of the block after block_argmax.
template <typename T>
__device__ __forceinline__ void record_and_factor(BlkWork<T>& w, int64_t n,
                                                  int64_t s, PivotKey k,
                                                  bool bad, T vs,
                                                  int* shstatus)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        int st = kStatusOk;
        if (bad)
            st = kStatusNonfinite;
        else if (k.slot < 0 || k.value == 0.0)
            st = kStatusSingular;
        w.piv_pos[s] = k.slot;
        w.piv_val[s] = k.value;
        if (st == kStatusOk) {
            const int a = w.perm[s];
            w.perm[s] = w.perm[k.slot];
            w.perm[k.slot] = a;
        } else {
            w.state->bad_step = (int)s;
            w.state->status = st;
        }
        *shstatus = st;
    }
    __syncthreads();
    if (*shstatus != kStatusOk) return;
    const T p = (T)k.value;
    const int64_t l = k.slot;
    T* row = w.W + s * w.ldw;
    for (int64_t j = s + tid; j < n; j += kBlkThreads) {
        const T v = row[j];
        row[j] = (j == s) ? p : ((j == l) ? vs : v) / p;
    }
}

// The first row of a panel: its updates are complete (previous panels'
// trailing updates); find its pivot and factor it.
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_head(int64_t n, int64_t s, BlkWork<T> w)
{
    __shared__ PivotKey sh[kBlkThreads / kWave];
    __shared__ int shflag, shstatus;
    __shared__ T shv;
    if (w.state->status != kStatusOk) return;
    const T* row = w.W + s * w.ldw;
    PivotKey k = no_candidate();
    bool bad = false;
    for (int64_t j = s + threadIdx.x; j < n; j += kBlkThreads) {
        const T v = row[j];
        if (j == s) shv = v;
        if (!offer(k, (double)v, w.perm[j], (int)j)) bad = true;
    }
    k = block_argmax<kBlkThreads>(k, bad, sh, &shflag);
    record_and_factor(w, n, s, k, bad, shv, &shstatus);
}

// Step s of the panel [s0, pend): exchange positions s and l in the earlier
// panel rows, then for each panel row i > s (one block each):
//   c = a_il; a_il <- a_is; a_is <- c;  a_ij <- a_ij - c * r_j  (j > s)
// Block 0 owns row s+1 and, when it is in the panel, finds and factors the
// next pivot.
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_step(int64_t n, int64_t s, int64_t s0, int64_t pend, BlkWork<T> w)
{
    __shared__ PivotKey sh[kBlkThreads / kWave];
    __shared__ int shflag, shstatus;
    __shared__ T shc, shv;
    if (w.state->status != kStatusOk) return;
    const int tid = threadIdx.x;
    const int64_t l = w.piv_pos[s];
    T* __restrict__ W = w.W;
    const int64_t ldw = w.ldw;
    if (blockIdx.x == 0 && l != s) {
        for (int64_t u = s0 + tid; u < s; u += kBlkThreads) {
            T* ru = W + u * ldw;
            const T a = ru[s];
            const T b = ru[l];
            ru[s] = b;
            ru[l] = a;
        }
    }
    const int64_t i = s + 1 + blockIdx.x;
    if (i >= pend) return;
    const T* rs = W + s * ldw; // factored pivot row s
    T* ri = W + i * ldw;
    if (tid == 0) shc = ri[l];
    __syncthreads(); // the multiplier is read before position l changes
    const T c = shc;
    const bool look = (blockIdx.x == 0);
    PivotKey k = no_candidate();
    bool bad = false;
    for (int64_t j = s + 1 + tid; j < n; j += kBlkThreads) {
        T x;
        if (j == l) {
            x = ri[s];
            ri[s] = c;
        } else {
            x = ri[j];
        }
        const T y = fma(-c, rs[j], x);
        ri[j] = y;
        if (look) {
            if (j == s + 1) shv = y;
            if (!offer(k, (double)y, w.perm[j], (int)j)) bad = true;
        }
    }
    if (!look) return;
    k = block_argmax<kBlkThreads>(k, bad, sh, &shflag);
    record_and_factor(w, n, s + 1, k, bad, shv, &shstatus);
}

// For the rows below the panel, where did each moved column come from?
// Position s0+t exchanged contents with position l_t at step s0+t, so the
// source of a destination is found by undoing the exchanges in reverse.
__global__ void __launch_bounds__(kBlkThreads)
blk_perm(int64_t s0, int nb, const int* __restrict__ piv_pos, int* colsrc,
         int* srcp, int* moved, const DevState* state)
{
    __shared__ int lp[kMaxPanel];
    if (state->status != kStatusOk) return;
    const int tid = threadIdx.x;
    for (int t = tid; t < kMaxPanel; t += kBlkThreads) {
        const int d = moved[t];
        if (d >= 0) {
            colsrc[d] = d;
            moved[t] = -1;
        }
    }
    for (int t = tid; t < nb; t += kBlkThreads) lp[t] = piv_pos[s0 + t];
    __syncthreads();
    const int64_t pend = s0 + nb;
    auto trace = [&](int64_t d) -> int {
        int64_t pos = d;
        for (int u = nb - 1; u >= 0; --u) {
            const int64_t a = s0 + u, b = lp[u];
            if (pos == a)
                pos = b;
            else if (pos == b)
                pos = a;
        }
        return (int)pos;
    };
    for (int t = tid; t < nb; t += kBlkThreads) {
        srcp[t] = trace(s0 + t);
        const int64_t d = lp[t];
        if (d >= pend) {
            colsrc[d] = trace(d);
            moved[t] = (int)d;
        }
    }
}

// L21 = A21 * U11^{-1}: for each row below the panel, x solves x U11 = a
// with a_t = W[i][srcp[t]] and U11 the unit upper triangle of the factored
// panel rows:  x_t = a_t - sum_{u<t} x_u U11[u][t].  Four lanes share a
// row (lane q handles u = q mod 4); U11 is packed by columns in LDS.
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_trsm(int64_t n, int64_t s0, int nb, BlkWork<T> w)
{
    extern __shared__ unsigned char smem_raw[];
    T* us = reinterpret_cast<T*>(smem_raw);
    const int packed = nb * (nb - 1) / 2;
    T* xs = us + packed;
    const int ldx = nb + 1;
    if (w.state->status != kStatusOk) return;
    const int tid = threadIdx.x;
    const T* __restrict__ W = w.W;
    const int64_t ldw = w.ldw;
    for (int e = tid; e < nb * nb; e += kBlkThreads) {
        const int u = e / nb, t = e - u * nb;
        if (u < t) us[t * (t - 1) / 2 + u] = W[(s0 + u) * ldw + s0 + t];
    }
    const int64_t pend = s0 + nb;
    const int r = tid >> 2, q = tid & 3;
    const int64_t i = pend + (int64_t)blockIdx.x * kTrsmRows + r;
    const bool valid = i < n;
    T* x = xs + r * ldx;
    if (valid)
        for (int u = q; u < nb; u += 4) x[u] = W[i * ldw + w.srcp[u]];
    __syncthreads();
    for (int t = 0; t < nb; ++t) {
        const T* ut = us + (t * (t - 1)) / 2;
        T part = 0;
        if (valid)
            for (int u = q; u < t; u += 4) part = fma(x[u], ut[u], part);
        part += __shfl_xor(part, 1, kWave);
        part += __shfl_xor(part, 2, kWave);
        if (valid && q == (t & 3)) x[t] -= part;
    }
    if (valid) {
        T* out = w.L + (i - pend) * w.ldl;
        for (int u = q; u < nb; u += 4) out[u] = x[u];
    }
}

// Compensated sum of log|p_s|; sign = prod sgn(p_s) * (-1)^(exchanges).
__global__ void __launch_bounds__(kBlkThreads)
blk_finalize(int64_t n, const int* __restrict__ piv_pos,
             const double* __restrict__ piv_val, const DevState* state,
             mc_result* out)
{
    __shared__ double ssum[kBlkThreads], scomp[kBlkThreads];
    __shared__ int spar[kBlkThreads];
    const int tid = threadIdx.x;
    const int st = state->status;
    if (st != kStatusOk) {
        if (tid == 0) {
            const bool sing = st == kStatusSingular;
            out->logabsdet = sing ? -INFINITY : NAN;
            out->sign = 0.0;
            out->info = sing ? (int64_t)state->bad_step + 1
                             : (int64_t)MC_INFO_NONFINITE;
        }
        return;
    }
    Compensated acc{0.0, 0.0};
    int parity = 0;
    for (int64_t s = tid; s < n; s += kBlkThreads) {
        const double p = piv_val[s];
        comp_add(acc, log(fabs(p)));
        parity ^= (p < 0.0) ? 1 : 0;
        parity ^= (piv_pos[s] != (int)s) ? 1 : 0;
    }
    ssum[tid] = acc.sum;
    scomp[tid] = acc.comp;
    spar[tid] = parity;
    __syncthreads();
    if (tid == 0) {
        Compensated tot{0.0, 0.0};
        int par = 0;
        for (int t = 0; t < kBlkThreads; ++t) {
            comp_merge(tot, Compensated{ssum[t], scomp[t]});
            par ^= spar[t];
        }
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

// ---------------------------------------------------------------- host side

template <typename T>
static size_t trsm_lds_bytes(int nb)
{
    return sizeof(T) * ((size_t)nb * (nb - 1) / 2 + (size_t)kTrsmRows * (nb + 1));
}

template <typename T>
hipError_t launch_blocked(const T* A, int64_t n, int64_t lda, int64_t b,
                          int update, BlkWork<T> w, mc_result* out,
                          hipStream_t stream)
{
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&blk_trsm<T>),
            hipFuncAttributeMaxDynamicSharedMemorySize,
            (int)trsm_lds_bytes<T>((int)kMaxPanel));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(blk_init<T>, dim3((unsigned)n), dim3(kBlkThreads), 0,
                       stream, A, lda, n, w);
    for (int64_t s0 = 0; s0 < n; s0 += b) {
        const int nb = (int)std::min<int64_t>(b, n - s0);
        const int64_t pend = s0 + nb;
        hipLaunchKernelGGL(blk_head<T>, dim3(1), dim3(kBlkThreads), 0, stream,
                           n, s0, w);
        for (int64_t s = s0; s < pend; ++s) {
            const int64_t blocks = std::max<int64_t>(1, pend - 1 - s);
            hipLaunchKernelGGL(blk_step<T>, dim3((unsigned)blocks),
                               dim3(kBlkThreads), 0, stream, n, s, s0, pend,
                               w);
        }
        if (pend >= n) break;
        const int64_t rows = n - pend;
        hipLaunchKernelGGL(blk_perm, dim3(1), dim3(kBlkThreads), 0, stream, s0,
                           nb, w.piv_pos, w.colsrc, w.srcp, w.moved, w.state);
        hipLaunchKernelGGL(blk_trsm<T>,
                           dim3((unsigned)((rows + kTrsmRows - 1) / kTrsmRows)),
                           dim3(kBlkThreads), trsm_lds_bytes<T>(nb), stream, n,
                           s0, nb, w);
        GemmArgs<T> g;
        g.C = w.W;
        g.ldc = w.ldw;
        g.r0 = pend;
        g.c0 = pend;
        g.M = rows;
        g.N = rows;
        g.K = nb;
        g.L = w.L;
        g.ldl = w.ldl;
        g.U = w.W + s0 * w.ldw;
        g.ldu = w.ldw;
        g.colsrc = w.colsrc;
        g.state = w.state;
        const ProfMark pm = prof_begin(stream);
        const hipError_t e = launch_trailing_update(g, update, stream);
        if (e != hipSuccess) return e;
        const double flops = 2.0 * (double)rows * (double)rows * nb;
        const double bytes = (double)sizeof(T) *
                             (2.0 * rows * rows + 2.0 * rows * nb);
        prof_end(stream, pm, 1, bytes, flops);
    }
    hipLaunchKernelGGL(blk_finalize, dim3(1), dim3(kBlkThreads), 0, stream, n,
                       w.piv_pos, w.piv_val, w.state, out);
    return hipGetLastError();
}

template hipError_t launch_blocked<double>(const double*, int64_t, int64_t,
                                           int64_t, int, BlkWork<double>,
                                           mc_result*, hipStream_t);
template hipError_t launch_blocked<float>(const float*, int64_t, int64_t,
                                          int64_t, int, BlkWork<float>,
                                          mc_result*, hipStream_t);

} // namespace mc
