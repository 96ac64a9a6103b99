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
// Per panel:
//   blk_panel_split  all b steps on one XCD, the panel's columns split over
//              its compute units (the default while the width fits: 8192
//              columns for FP64 panels of 128 rows, 16384 otherwise);
//              otherwise a row-per-block chain (blk_head_r + blk_panel_x or
//              blk_panel, then blk_fixup_x / blk_fixup and blk_perm), or one
//              launch per step (blk_head, blk_step)
//   blk_trsm_mfma  L21 = gather(A21) * U11^{-1} on the matrix cores
//   gemm       A22 <- gather(A22) - L21 * U12 (mc_gemm.hip): with lookahead
//              the next panel's rows first, the rest on a side stream beside
//              the next panel
#include <algorithm>
#include <type_traits>
#include <atomic>
#include <mutex>

#include "mc_device.h"
#include "mc_gemm.h"
#include "mc_internal.h"
#include "mc_mfma.h"

namespace mc {

constexpr int kBlkThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_init(const T* __restrict__ A, int64_t lda, int64_t n, BlkWork<T> w)
{
    const int64_t i = blockIdx.x;
    if (A != w.W) // in-place factorisation: the caller's matrix is W
        for (int64_t j = threadIdx.x; j < n; j += kBlkThreads)
            w.W[i * w.ldw + j] = A[i * lda + j];
    if (i == 0) {
        for (int64_t j = threadIdx.x; j < n; j += kBlkThreads) {
            w.perm[j] = (int)j;
            w.colsrc[j] = (int)j;
            w.colsrc_b[j] = (int)j;
        }
        for (int t = threadIdx.x; t < kMaxPanel; t += kBlkThreads) {
            w.moved[t] = -1;
            w.moved_b[t] = -1;
        }
        // no candidate record of an earlier factorisation may pass for one
        // of this one
        for (int t = threadIdx.x; t < 4 * kSplitSlices; t += kBlkThreads) w.xrec[t] = 0;
        if (threadIdx.x == 0) {
            w.state->status = kStatusOk;
            w.state->bad_step = 0;
            w.claim[0] = 0;
            w.claim[1] = -1;
            w.claim[2] = 0;
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

// ---- register-resident step kernels (rows up to kStepThreads * 16 wide) ----
//
// One block of kStepThreads threads per row; thread t holds the entries at
// positions j0 + t + e * kStepThreads, e < EPT, in registers.  Every load is
// issued before the block's single barrier, so a step costs about one memory
// latency plus the argmax reduction.

constexpr int kStepThreads = 1024;

// Decide the step's status from the reduced key (same on every thread).
__device__ __forceinline__ int pivot_status(const PivotKey& k, bool bad)
{
    if (bad) return kStatusNonfinite;
    if (k.slot < 0 || k.value == 0.0) return kStatusSingular;
    return kStatusOk;
}

// Thread 0's bookkeeping for the pivot of step s (runs beside the
// factoring stores of the other threads).
template <typename T>
__device__ __forceinline__ void record_pivot(BlkWork<T>& w, int64_t s,
                                             const PivotKey& k, int st)
{
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
}

// Write row s (values y[] at positions s + tid + e*NT) in factored form.
template <typename T, int EPT>
__device__ __forceinline__ void store_factored(T* row, int64_t s, int64_t n,
                                               const T (&y)[EPT], T p,
                                               int64_t l, T vs)
{
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s + threadIdx.x + (int64_t)e * kStepThreads;
        if (j < n) row[j] = (j == s) ? p : ((j == l) ? vs : y[e]) / p;
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kStepThreads)
blk_head_r(int64_t n, int64_t s, BlkWork<T> w)
{
    __shared__ PivotKey sh[kStepThreads / kWave];
    __shared__ int shflag, shpc;
    __shared__ T shv;
    // the panel starting here has not published any later step yet
    for (int t = threadIdx.x; t < kMaxPanel; t += kStepThreads) w.stepflag[t] = 0;
    if (threadIdx.x == 0) {
        w.claim[0] = 0;
        w.claim[1] = -1;
    }
    if (w.state->status != kStatusOk) return;
    T* row = w.W + s * w.ldw;
    T y[EPT];
    int pc[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s + threadIdx.x + (int64_t)e * kStepThreads;
        if (j < n) {
            y[e] = row[j];
            pc[e] = w.perm[j];
        }
    }
    if (threadIdx.x == 0) {
        shv = y[0];
        shpc = pc[0];
    }
    PivotKey k = no_candidate();
    bool bad = false;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s + threadIdx.x + (int64_t)e * kStepThreads;
        if (j < n && !offer(k, (double)y[e], pc[e], (int)j)) bad = true;
    }
    k = block_argmax<kStepThreads>(k, bad, sh, &shflag);
    const int st = pivot_status(k, bad);
    if (threadIdx.x == 0) record_pivot(w, s, k, st);
    if (st != kStatusOk) return;
    store_factored<T, EPT>(row, s, n, y, (T)k.value, k.slot, shv);
    // the column ids after this step's exchange, for the single-XCD panel
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s + threadIdx.x + (int64_t)e * kStepThreads;
        if (j < n) w.perm0[j] = (j == s) ? k.colid : ((j == k.slot) ? shpc : pc[e]);
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kStepThreads)
blk_step_r(int64_t n, int64_t s, int64_t s0, int64_t pend, BlkWork<T> w)
{
    __shared__ PivotKey sh[kStepThreads / kWave];
    __shared__ int shflag;
    __shared__ T shv;
    if (w.state->status != kStatusOk) return;
    const int tid = threadIdx.x;
    const int64_t l = w.piv_pos[s];
    T* __restrict__ W = w.W;
    const int64_t ldw = w.ldw;
    if (blockIdx.x == 0 && l != s) {
        for (int64_t u = s0 + tid; u < s; u += kStepThreads) {
            T* ru = W + u * ldw;
            const T a = ru[s];
            const T b = ru[l];
            ru[s] = b;
            ru[l] = a;
        }
    }
    const int64_t i = s + 1 + blockIdx.x;
    if (i >= pend) return;
    const T* rs = W + s * ldw;
    T* ri = W + i * ldw;
    const bool look = (blockIdx.x == 0);
    // every load first: the multiplier, the row, the pivot row, column ids
    const T c = ri[l];
    T x[EPT], r[EPT];
    int pc[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s + 1 + tid + (int64_t)e * kStepThreads;
        if (j < n) {
            x[e] = ri[(j == l) ? s : j];
            r[e] = rs[j];
            if (look) pc[e] = w.perm[j];
        }
    }
    __syncthreads(); // no position of row i is written before all reads
    T y[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) y[e] = fma(-c, r[e], x[e]);
    if (tid == 0 && l != s) ri[s] = c; // the multiplier moves to position s
    if (!look) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t j = s + 1 + tid + (int64_t)e * kStepThreads;
            if (j < n) ri[j] = y[e];
        }
        return;
    }
    if (tid == 0) shv = y[0];
    PivotKey k = no_candidate();
    bool bad = false;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s + 1 + tid + (int64_t)e * kStepThreads;
        if (j < n && !offer(k, (double)y[e], pc[e], (int)j)) bad = true;
    }
    k = block_argmax<kStepThreads>(k, bad, sh, &shflag);
    const int st = pivot_status(k, bad);
    if (tid == 0) record_pivot(w, s + 1, k, st);
    if (st != kStatusOk) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t j = s + 1 + tid + (int64_t)e * kStepThreads;
            if (j < n) ri[j] = y[e];
        }
        return;
    }
    store_factored<T, EPT>(ri, s + 1, n, y, (T)k.value, k.slot, shv);
}

// ---- persistent panel: one launch per panel, rows held in registers ----
//
// Block r owns panel row i = s0 + 1 + r and keeps positions s0 .. n-1 of it
// in registers for the whole panel (thread t holds s0 + t + e*kStepThreads).
// For each step s < i it waits until the pivot row s is published (thread 0
// spins on stepflag with an agent-scope acquire, bounded), reads r = row s
// from memory, exchanges the multiplier c (position l) and the entry at
// position s through LDS, and applies
//     a_il <- a_is - c r_l,  a_is <- c,  a_ij <- a_ij - c r_j  (j > s, j != l)
// The block whose row is the next pivot row finds the pivot, writes its row
// in factored form, records the pivot and publishes it (release).  Rows
// published earlier still need the exchanges of later steps; blk_perm's
// fix-up blocks apply them after the panel.
//
// Every inter-block wait is bounded by one second of the 100 MHz real-time
// counter (a panel step takes microseconds): a wait that runs out marks the
// factorisation aborted and the kernel drains instead of hanging.
constexpr uint64_t kWaitTicks = 100000000ull;

__device__ __forceinline__ uint64_t now_ticks()
{
    return __builtin_amdgcn_s_memrealtime();
}

// Relaxed device-scope load: coherent across the XCDs' L2 caches without a
// fence (used for everything another block published during the kernel).
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s_waitcnt vmcnt(0) (gfx9 encoding; expcnt and lgkmcnt left at their
// maxima): every vector memory access of this wavefront has completed.
constexpr int kWaitVmcnt0 = 0x0F70;

template <typename T, int EPT>
__global__ void __launch_bounds__(kStepThreads)
blk_panel(int64_t n, int64_t s0, int64_t pend, BlkWork<T> w)
{
    __shared__ PivotKey sh[kStepThreads / kWave];
    __shared__ int shflag;
    __shared__ T sh_c, sh_xs, sh_vi; // sh_vi: own row at position i (never
                                     // shares a slot with the last step)
    __shared__ int sh_status;
    const int tid = threadIdx.x;
    const int64_t i = s0 + 1 + blockIdx.x; // this block's row
    T* ri = w.W + i * w.ldw;
    T v[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s0 + tid + (int64_t)e * kStepThreads;
        if (j < n) v[e] = ri[j];
    }
    for (int64_t s = s0; s < i; ++s) {
        if (s > s0 && tid == 0) {
            long spins = 0;
            const uint64_t t0 = now_ticks();
            // poll with device-coherent loads and no acquire fence (a fence
            // per poll would invalidate this XCD's L2 under every block)
            while (__hip_atomic_load(&w.stepflag[s - s0], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) == 0) {
                ++spins;
                if ((spins & 255) == 0 && now_ticks() - t0 > kWaitTicks) {
                    __hip_atomic_store(&w.state->status, (int)kStatusAborted,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                if ((spins & 1023) == 0 &&
                    __hip_atomic_load(&w.state->status, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) != kStatusOk)
                    break; // another block stopped the factorisation
                __builtin_amdgcn_s_sleep(1);
            }
            sh_status = __hip_atomic_load(&w.state->status, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        }
        if (s == s0 && tid == 0) sh_status = w.state->status;
        __syncthreads();
        if (sh_status != kStatusOk) return; // uniform across the block
        // the published row and pivot are read with device-coherent loads
        // (no acquire fence: that would invalidate this XCD's whole L2)
        const int64_t l = ld_agent(&w.piv_pos[s]);
        const T* rs = w.W + s * w.ldw;
        T r[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t j = s0 + tid + (int64_t)e * kStepThreads;
            r[e] = (j > s && j < n) ? ld_agent(&rs[j]) : T(0);
            if (j == l) sh_c = v[e];
            if (j == s) sh_xs = v[e];
        }
        __syncthreads();
        const T c = sh_c, xs = sh_xs;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int64_t j = s0 + tid + (int64_t)e * kStepThreads;
            if (j == s)
                v[e] = c;
            else if (j > s && j < n)
                v[e] = fma(-c, r[e], (j == l) ? xs : v[e]);
        }
    }
    // row i is now final: find its pivot, factor it, publish it
    if (i + 1 > pend) return;
    int cid[EPT]; // original column ids, all requested before any is used
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s0 + tid + (int64_t)e * kStepThreads;
        cid[e] = (j >= i && j < n) ? ld_agent(&w.perm[j]) : 0;
    }
    PivotKey k = no_candidate();
    bool bad = false;
    int cid_i = 0; // original column at position i (thread owning j == i)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s0 + tid + (int64_t)e * kStepThreads;
        if (j >= i && j < n && !offer(k, (double)v[e], cid[e], (int)j))
            bad = true;
        if (j == i) {
            sh_vi = v[e];
            cid_i = cid[e];
        }
    }
    k = block_argmax<kStepThreads>(k, bad, sh, &shflag);
    const int st = pivot_status(k, bad);
    const T p = (T)k.value, vi = sh_vi;
    // publish with device-scope (write-through) stores, wait until every
    // one is acknowledged, then raise the flag: no cache-wide write-back
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t j = s0 + tid + (int64_t)e * kStepThreads;
        if (j >= n) continue;
        T out = v[e];
        if (st == kStatusOk && j >= i)
            out = (j == i) ? p : ((j == k.slot) ? vi : v[e]) / p;
        st_agent(&ri[j], out);
        if (st == kStatusOk && j == i) { // exchange the column ids
            st_agent(&w.perm[i], k.colid);
            st_agent(&w.perm[k.slot], cid_i);
        }
    }
    if (tid == 0) {
        st_agent(&w.piv_pos[i], k.slot);
        st_agent(&w.piv_val[i], k.value);
        if (st != kStatusOk) {
            st_agent(&w.state->bad_step, (int)i);
            st_agent(&w.state->status, st);
        }
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (tid == 0)
        __hip_atomic_store(&w.stepflag[i - s0], 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---- single-XCD persistent panel ----
//
// The same algorithm as blk_panel, confined to the compute units of one XCD
// so that the blocks exchange the published rows through that XCD's shared
// L2: stores are plain (they land in L2), a vmcnt(0) wait orders them before
// the flag, and readers use loads with the sc0+nt policy, which re-fetch
// from the L2 even when the line sits in the reader's L1 (measured on
// gfx950: an sc0-only load keeps returning a stale L1 line, and a plain
// store is never seen from another XCD by any load policy).
//
// The grid is launched eight times over (blocks go to the XCDs in turn);
// block 0 elects its XCD and the blocks that land there claim slots.  Slot q
// owns the panel rows s0+1+q, s0+1+q+S, ... (S slots, at most R rows each),
// all held in registers from the start, so every published row is read once
// per block and applied to all of its rows: the chain of a step is one flag,
// one row read, the pivot search and the publication.  All slots must be
// resident together (S <= 32, one block per compute unit of the XCD); every
// wait is bounded.

// L2-served loads (sc0 nt) through a buffer descriptor covering `bytes`
// from base (out-of-range offsets read as zero).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t l2_rsrc(const void* base,
                                                         int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                             (int)bytes, 0x00020000);
}

constexpr int kL2Policy = 3; // cache-policy operand: sc0 | nt

template <typename T>
__device__ __forceinline__ T l2_load(__amdgpu_buffer_rsrc_t r, int index);

template <>
__device__ __forceinline__ double l2_load<double>(__amdgpu_buffer_rsrc_t r,
                                                  int index)
{
    return __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(r, index * 8, 0, kL2Policy));
}

template <>
__device__ __forceinline__ float l2_load<float>(__amdgpu_buffer_rsrc_t r,
                                                int index)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(r, index * 4, 0, kL2Policy));
}

template <>
__device__ __forceinline__ int l2_load<int>(__amdgpu_buffer_rsrc_t r,
                                            int index)
{
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, index * 4, 0, kL2Policy);
}

// Polling form: the empty asm with a memory clobber keeps the compiler
// from hoisting or merging the load (the volatile bit of the buffer
// intrinsics would instead raise the scope to system, past the L2).
__device__ __forceinline__ int l2_poll(__amdgpu_buffer_rsrc_t r, int index)
{
    asm volatile("" ::: "memory");
    return l2_load<int>(r, index);
}

// Scratch of the single-XCD panel's pivot search (one entry per wavefront).
struct PanelXShared {
    double wmax[16];
    int wbad[16];
    unsigned long long wkey[16];
    double piv_p;   // the published row's pivot (0 when the step failed)
    double piv_vi;  // the published row's entry at its own position i
    int piv_l;      // the pivot position (-1 when the step failed)
};

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, kWave));
    return x;
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long x)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long y = __shfl_xor(x, off, kWave);
        x = y < x ? y : x;
    }
    return x;
}

// Entry e (wave-uniform, < EPT) of a register array, for the one thread
// that owns a given position: a chain of selects that starts from a
// constant (a select between two array loads could be folded into one
// load at a computed address, which would move the array to scratch).
template <typename T, int EPT>
__device__ __forceinline__ T pick(const T (&a)[EPT], int e)
{
    T r = T(0);
#pragma unroll
    for (int q = 0; q < EPT; ++q) r = (q == e) ? a[q] : r;
    return r;
}

template <typename T, int EPT>
__device__ __forceinline__ void put(T (&a)[EPT], int e, T v)
{
#pragma unroll
    for (int q = 0; q < EPT; ++q) a[q] = (q == e) ? v : a[q];
}

// Update of one panel row x by step s (pivot position l): every entry right
// of s takes -c times the factored pivot row, the row's entry at l (the
// multiplier c) is stashed at s (Figure 6, step 4.8) and position l takes
// the row's old entry at s, xs, minus c times the pivot row's entry there.
// r holds the pivot row with zeros at positions <= s and >= n, so one fma
// per entry does the bulk; the threads owning s and l then set those two.
// The pivot row arrives unfactored (entries v_j, pivot p): cp = c / p, and
// the factored entry at l is the pivot row's entry at s (atl); the panel's
// first row arrives factored: cp = c, atl = its entry at l.
template <typename T, int NT, int EPT>
__device__ __forceinline__ void panelx_apply(T (&x)[EPT], const T (&r)[EPT],
                                             int s0, int s, int l, T c, T cp,
                                             T xs, bool factored, T vs)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int e = 0; e < EPT; ++e) x[e] = fma(-cp, r[e], x[e]);
    if (tid == (l - s0) % NT) { // owner of position l (l >= s)
        const int el = (l - s0) / NT;
        put<T, EPT>(x, el, fma(-cp, factored ? pick<T, EPT>(r, el) : vs, xs));
    }
    if (tid == (s - s0) % NT) put<T, EPT>(x, (s - s0) / NT, c);
}

// Publication of panel row i held in v (single-XCD panel): the row goes out
// unfactored first (the stores drain while the pivot is searched), then the
// pivot (largest |v| over positions >= i, ties to the smallest original
// column id, Section 2.2), the column-id exchange, and the flag, which
// carries the pivot position + 1.  On return sm.piv_l / piv_p / piv_vi hold
// the pivot position (-1 if the step failed), its value and the row's entry
// at i, for the block's own next rows.  ids[j - s0] is the original column id at
// position j.  Thread tid holds positions s0 + e*NT + tid; position tests
// compare tid with wave-uniform bounds, so no per-entry index is kept in a
// vector register (n <= 2^30: 32-bit indices).
template <typename T, int NT, int EPT>
__device__ __forceinline__ void panelx_publish(int n, int s0, int i, const T (&v)[EPT],
                                               const int* ids, PanelXShared& sm,
                                               const BlkWork<T>& w)
{
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    T* ri = w.W + (int64_t)i * w.ldw + s0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        if (tid < n - s0 - e * NT) ri[e * NT + tid] = v[e];
        if (tid == i - s0 - e * NT) sm.piv_vi = (double)v[e];
    }
    // pass 1: the largest |v| and whether any entry is not finite
    double m = 0.0;
    bool bad = false;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int base = s0 + e * NT;
        const bool in = tid >= i - base && tid < n - base;
        const double a = fabs((double)v[e]);
        bad |= in && !isfinite(a);
        m = fmax(m, in ? a : 0.0);
    }
    m = wave_max(m);
    const bool wbad = __any(bad);
    if (lane == 0) {
        sm.wmax[wv] = m;
        sm.wbad[wv] = wbad;
    }
    __syncthreads();
    double M = sm.wmax[0];
    int anybad = sm.wbad[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
        M = fmax(M, sm.wmax[q]);
        anybad |= sm.wbad[q];
    }
    const int st = anybad ? kStatusNonfinite : (M > 0.0 ? kStatusOk : kStatusSingular);
    if (st == kStatusOk) { // uniform
        // pass 2: among the entries of magnitude M, the smallest column id;
        // key = id << 32 | sign << 31 | slot
        unsigned long long key = ~0ull;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int base = s0 + e * NT;
            if (tid >= i - base && tid < n - base && fabs((double)v[e]) == M) {
                const unsigned long long c =
                    ((unsigned long long)(unsigned)ids[e * NT + tid] << 32) |
                    ((unsigned long long)(v[e] < T(0)) << 31) |
                    (unsigned long long)(unsigned)(base + tid);
                key = c < key ? c : key;
            }
        }
        key = wave_min(key);
        if (lane == 0) sm.wkey[wv] = key;
        __syncthreads();
        if (tid == 0) {
            unsigned long long k = sm.wkey[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) k = sm.wkey[q] < k ? sm.wkey[q] : k;
            const int slot = (int)(k & 0x7fffffffu);
            const int colid = (int)(k >> 32);
            const double p = ((k >> 31) & 1u) ? -M : M;
            w.piv_pos[i] = slot;
            w.piv_val[i] = p;
            w.perm[slot] = ids[i - s0]; // exchange the column ids
            w.perm[i] = colid;
            sm.wkey[0] = (unsigned long long)(slot + 1);
            sm.piv_l = slot;
            sm.piv_p = p;
        }
    } else if (tid == 0) {
        w.piv_pos[i] = -1;
        w.piv_val[i] = 0.0;
        w.state->bad_step = i;
        w.state->status = st;
        sm.wkey[0] = 1;
        sm.piv_l = -1;
        sm.piv_p = 0.0;
    }
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0); // every store has reached L2
    __syncthreads();
    if (tid == 0) w.stepflag[i - s0] = (int)sm.wkey[0];
}

template <typename T, int NT, int EPT, int R>
__global__ void __launch_bounds__(NT)
blk_panel_x(int64_t n64, int64_t s064, int64_t pend64, int nslots, BlkWork<T> w)
{
    const int n = (int)n64, s0 = (int)s064, pend = (int)pend64;
    __shared__ PanelXShared sm;
    __shared__ int sh_status, sh_slot, sh_l;
    __shared__ T sh_c[R], sh_xs[R];
    __shared__ int sh_perm[NT * EPT]; // column ids of positions s0 ..
    const int tid = threadIdx.x;
    // block 0 publishes its XCD (device-coherent store); blocks on other
    // XCDs leave, the others claim slots from a counter in that XCD's L2
    if (tid == 0) {
        const int x = xcc_id();
        int e = x;
        if (blockIdx.x == 0) {
            st_agent(&w.claim[1], x);
        } else {
            const uint64_t t0 = now_ticks();
            while ((e = ld_agent(&w.claim[1])) < 0) {
                if (now_ticks() - t0 > kWaitTicks) {
                    st_agent(&w.state->status, (int)kStatusAborted);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        sh_slot = (e == x) ? 0 : -1;
    }
    __syncthreads();
    if (sh_slot < 0) return;
    const __amdgpu_buffer_rsrc_t flags = l2_rsrc(w.stepflag, sizeof(int) * kMaxPanel);
    const __amdgpu_buffer_rsrc_t pivs = l2_rsrc(w.piv_pos, sizeof(int) * (int64_t)n);
    const __amdgpu_buffer_rsrc_t pvals = l2_rsrc(w.piv_val, sizeof(double) * (int64_t)n);
    const __amdgpu_buffer_rsrc_t stat = l2_rsrc(&w.state->status, sizeof(int));
    for (;;) { // slots in increasing order until none is left
        __syncthreads();
        if (tid == 0) sh_slot = atomicAdd(&w.claim[0], 1);
        __syncthreads();
        const int slot = sh_slot;
        if (slot >= nslots) return;
        // this slot's rows: R consecutive panel rows, so it only ever waits
        // for rows of lower slots, which were claimed (and so are running
        // or done) before it
        int row[R]; // increasing; -1 once gone
        T v[R][EPT];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            row[q] = s0 + 1 + slot * R + q;
            if (row[q] >= pend) row[q] = -1;
            const T* rq = w.W + (int64_t)(row[q] < 0 ? 0 : row[q]) * w.ldw + s0;
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                v[q][e] = (row[q] >= 0 && tid < n - s0 - e * NT) ? rq[e * NT + tid] : T(0);
        }
        // the block's copy of the column ids, from the snapshot the head
        // step wrote (the live array changes while the panel runs); each
        // later step's exchange is applied here as it is taken
        for (int t = tid; t < n - s0; t += NT) sh_perm[t] = w.perm0[s0 + t];
        // phase A: the steps before this slot's first row, whose pivot
        // rows other blocks publish (the head step's row arrives factored)
        for (int s = s0; s < row[0]; ++s) {
            if (tid == 0) {
                int f = 1;
                if (s > s0) {
                    long spins = 0;
                    const uint64_t t0 = now_ticks();
                    while ((f = l2_poll(flags, s - s0)) == 0) {
                        ++spins;
                        if ((spins & 255) == 0) {
                            if (now_ticks() - t0 > kWaitTicks) {
                                w.state->status = kStatusAborted;
                                break;
                            }
                            if (l2_poll(stat, 0) != kStatusOk) break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                sh_status = l2_poll(stat, 0);
                sh_l = (s > s0) ? f - 1 : l2_load<int>(pivs, s);
            }
            __syncthreads();
            if (sh_status != kStatusOk) return; // uniform across the block
            const int l = __builtin_amdgcn_readfirstlane(sh_l);
            const bool factored = (s == s0);
            const T* rs = w.W + (int64_t)s * w.ldw;
            // the pivot row through a descriptor that starts at position
            // s+1: offsets below it wrap to huge values and, like those at
            // or past n, fail the range check and read as zero
            const __amdgpu_buffer_rsrc_t rrow =
                l2_rsrc(rs + s + 1, sizeof(T) * (int64_t)(n - s - 1));
            T r[EPT];
#pragma unroll
            for (int e = 0; e < EPT; ++e) r[e] = l2_load<T>(rrow, s0 + e * NT + tid - s - 1);
            T vs = T(0), ps = T(1);
            if (!factored) {
                vs = l2_load<T>(l2_rsrc(rs + s, sizeof(T)), 0);
                ps = (T)l2_load<double>(pvals, s);
            }
            if (tid == 0 && !factored && l != s) { // step s exchanged l and s
                const int a = sh_perm[s - s0];
                sh_perm[s - s0] = sh_perm[l - s0];
                sh_perm[l - s0] = a;
            }
            if (tid == (l - s0) % NT) { // owner of position l: multipliers
                const int el = (l - s0) / NT;
#pragma unroll
                for (int q = 0; q < R; ++q) sh_c[q] = pick<T, EPT>(v[q], el);
            }
            if (tid == (s - s0) % NT) { // owner of position s
                const int es = (s - s0) / NT;
#pragma unroll
                for (int q = 0; q < R; ++q) sh_xs[q] = pick<T, EPT>(v[q], es);
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (row[q] < 0) continue;
                const T c = sh_c[q];
                panelx_apply<T, NT, EPT>(v[q], r, s0, s, l, c, factored ? c : c / ps,
                                         sh_xs[q], factored, vs);
            }
        }
        // phase B: this slot's rows in order; each is final once the
        // previous one is applied, which the block does from registers
        for (;;) {
            const int i = row[0];
            panelx_publish<T, NT, EPT>(n, s0, i, v[0], sh_perm, sm, w);
            const int l = sm.piv_l;
            if (l < 0) return; // the step failed; its status is published
            const int next = (R > 1) ? row[R > 1 ? 1 : 0] : -1;
            if (next < 0) break;
            const T p = (T)sm.piv_p, vi = (T)sm.piv_vi;
            if (tid == 0 && l != i) { // step i exchanged l and i
                const int a = sh_perm[i - s0];
                sh_perm[i - s0] = sh_perm[l - s0];
                sh_perm[l - s0] = a;
            }
            if (tid == (l - s0) % NT) {
                const int el = (l - s0) / NT;
#pragma unroll
                for (int q = 1; q < R; ++q) sh_c[q] = pick<T, EPT>(v[q], el);
            }
            if (tid == (i - s0) % NT) {
                const int ei = (i - s0) / NT;
#pragma unroll
                for (int q = 1; q < R; ++q) sh_xs[q] = pick<T, EPT>(v[q], ei);
            }
            __syncthreads();
            T r[EPT]; // the published row right of i, zero elsewhere
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int base = s0 + e * NT;
                r[e] = (tid > i - base && tid < n - base) ? v[0][e] : T(0);
            }
#pragma unroll
            for (int q = 1; q < R; ++q) {
                if (row[q] < 0) continue;
                const T c = sh_c[q];
                panelx_apply<T, NT, EPT>(v[q], r, s0, i, l, c, c / p, sh_xs[q],
                                         false, vi);
            }
#pragma unroll
            for (int q = 0; q + 1 < R; ++q) {
                row[q] = row[q + 1];
#pragma unroll
                for (int e = 0; e < EPT; ++e) v[q][e] = v[q + 1][e];
            }
            row[R - 1] = -1;
        }
    }
}

// Undo the exchanges of panel steps hi-1 down to lo (step t exchanged
// positions s0+t and lp[t]) on Q positions per lane at once.  lp0 and lp1
// hold lp[lane] and lp[lane + 64]; every step's partner is read from them
// with readlane (lo, hi and the step index are wave-uniform).
template <int Q>
__device__ __forceinline__ void undo_exchanges(int (&pos)[Q], int s0, int lo,
                                               int hi, int lp0, int lp1)
{
    for (int t = hi - 1; t >= lo; --t) {
        const int b = t < kWave ? __builtin_amdgcn_readlane(lp0, t)
                                : __builtin_amdgcn_readlane(lp1, t - kWave);
        const int a = s0 + t;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            pos[q] = pos[q] == a ? b : (pos[q] == b ? a : pos[q]);
    }
}

// ---- column-split panel (one XCD) ----
//
// For panels at most kSplitSlices * 256 positions wide.  P blocks on one
// XCD split the panel's positions into slices of CP = 8 * CPW columns and
// keep their slice of all nb panel rows in registers for the whole panel:
// wave v holds columns v*CPW .. v*CPW+CPW-1 of the slice, lane L the rows L
// and L + 64.  Columns are never moved in memory: each keeps its original
// id and tracks its current position, and the exchange of a step (the pivot
// column and the column at the step's own position, Section 2.4) only swaps
// two positions.  Step k (row k of the panel, absolute step s = s0 + k):
//   1. every block applies step k-1 to the half of its rows that holds row
//      k and finds its best entry of row k (largest |a|, ties to the
//      smallest original id, Section 2.2);
//   2. the wave holding that column posts it: the column's entries of the
//      panel rows (with step k-1 applied), then one 16-byte record
//      {|a| | generation bit, tag | sign | non-finite | id | position};
//   3. every block reads the P records, takes the same winner, reads the
//      winner's column c and keeps c_i / p as the multipliers of step k;
//      the winning column retires (its entries below row k are the
//      multipliers of Figure 6 step 4.8 and stay as they are);
//   4. the rest of step k-1 (the other half of the rows) is applied while
//      the records are awaited.
// The update of an active column j is a_ij <- a_ij - (c_i / p) a_kj for the
// rows i > k (Eq. 2/3 with the factored pivot row written out).  After the
// last step every block writes its slice at the columns' final positions:
// row i divided by its pivot at the columns that were still active at step
// i (the factored rows of Section 2.3), the pivot itself and the
// multipliers as they are.  All P blocks must be resident together (one
// per compute unit of the XCD); every wait is bounded.

constexpr int kSplitThreads = 512;
constexpr int kSplitWaves = kSplitThreads / kWave;
constexpr int kSplitNone = 0x7fffffff; // a column no step of the panel took

static std::atomic<bool> g_split_on{true};

int split_panel_set(int on) { return g_split_on.exchange(on != 0) ? 1 : 0; }

// Largest |a| first, then the smaller key (original id in the high word).
__device__ __forceinline__ void split_take(uint64_t& a, uint64_t& k, uint64_t oa,
                                           uint64_t ok)
{
    const bool t = oa > a || (oa == a && ok < k);
    a = t ? oa : a;
    k = t ? ok : k;
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t x, uint64_t ident)
{
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)ident, (int)(uint32_t)x,
                                               CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(ident >> 32),
                                               (int)(uint32_t)(x >> 32), CTRL,
                                               ROWMASK, 0xf, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ void best_step(uint64_t& a, uint64_t& k)
{
    const uint64_t oa = dpp64<CTRL, ROWMASK>(a, 0ull);
    const uint64_t ok = dpp64<CTRL, ROWMASK>(k, ~0ull);
    split_take(a, k, oa, ok);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// The best (a, k) over the 64 lanes, in every lane: row shifts 1, 2, 4, 8
// leave each row's best in its lane 15, the two row broadcasts carry them
// to lane 63.  Called with every lane active.
__device__ __forceinline__ void wave_best(uint64_t& a, uint64_t& k)
{
    best_step<0x111, 0xf>(a, k); // row_shr:1
    best_step<0x112, 0xf>(a, k); // row_shr:2
    best_step<0x114, 0xf>(a, k); // row_shr:4
    best_step<0x118, 0xf>(a, k); // row_shr:8
    best_step<0x142, 0xa>(a, k); // row_bcast:15
    best_step<0x143, 0xc>(a, k); // row_bcast:31
    a = readlane64(a, 63);
    k = readlane64(k, 63);
}

// Plain buffer access of the panel rows (voffset per lane, soffset uniform).
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int voff,
                                                  int soff)
{
    typedef unsigned int v2u32 __attribute__((__vector_size__(8)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u32, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, int voff,
                                                 int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

__device__ __forceinline__ double wave_uniform(double v)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Largest 32-bit value over the 64 lanes (every lane active), in every
// lane: the same row shifts and broadcasts as wave_best.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp_max_step(uint32_t x)
{
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xf, false);
    return x > o ? x : o;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x)
{
    x = dpp_max_step<0x111, 0xf>(x);
    x = dpp_max_step<0x112, 0xf>(x);
    x = dpp_max_step<0x114, 0xf>(x);
    x = dpp_max_step<0x118, 0xf>(x);
    x = dpp_max_step<0x142, 0xa>(x);
    x = dpp_max_step<0x143, 0xc>(x);
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// The best (a, k) of the wave (largest a, then smallest k), returned
// uniformly: the high words of a first, then, only where several lanes
// share the largest high word, the low words, and only for exact ties the
// keys.
__device__ __forceinline__ void wave_best_fast(uint64_t& a, uint64_t& k)
{
    const uint32_t hi = (uint32_t)(a >> 32);
    const uint32_t mhi = wave_max_u32(hi);
    uint64_t m = __builtin_amdgcn_ballot_w64(hi == mhi);
    if (__builtin_popcountll(m) > 1) {
        const bool in = hi == mhi;
        const uint32_t lo = in ? (uint32_t)a : 0u;
        const uint32_t mlo = wave_max_u32(lo);
        m = __builtin_amdgcn_ballot_w64(in && lo == mlo);
        if (__builtin_popcountll(m) > 1) { // exact ties: the smallest key
            uint64_t aa = (in && lo == mlo) ? a : 0ull;
            uint64_t kk = (in && lo == mlo) ? k : ~0ull;
            wave_best(aa, kk);
            a = aa;
            k = kk;
            return;
        }
    }
    const int l = __builtin_ctzll(m);
    a = readlane64(a, l);
    k = readlane64(k, l);
}

// Columns per pass of the LDS transposes that load and store a wavefront's
// columns (at most 32, so the buffer stays 64 x 33 per wavefront).
template <int CPW>
constexpr int split_tc()
{
    return CPW < 32 ? CPW : 32;
}

template <typename T, int CPW>
static size_t split_lds_bytes()
{
    return sizeof(T) * (size_t)kSplitWaves * 64 * (split_tc<CPW>() + 1);
}

// H: halves of 64 rows the panel has (2 for up to 128 rows, 1 for up to 64).
template <typename T, int CPW, int H = 2>
__global__ void __launch_bounds__(kSplitThreads)
blk_panel_split(int64_t n64, int64_t s064, int nb, int nslices, int on_xcc0, BlkWork<T> w)
{
    constexpr int CP = kSplitWaves * CPW; // columns per slice
    constexpr int TC = split_tc<CPW>();   // columns per transpose pass
    constexpr int TBLD = TC + 1;
    extern __shared__ unsigned char smem_raw[];
    T* tb = reinterpret_cast<T*>(smem_raw); // [wave][64][TBLD] transposes
    __shared__ T prow[2][CP];               // row k of the slice, by step parity
    __shared__ T nrow[2][CP];               // row k+1 staged during step k
    __shared__ T mult[2][kMaxPanel];        // multipliers c_i / p, by step parity
    __shared__ double pv[kMaxPanel];        // pivot of each step
    __shared__ int pl[kMaxPanel];           // pivot position of each step
    __shared__ int cpos[CP], cstep[CP], cid[CP];
    __shared__ int invpos[kMaxPanel]; // panel position s0+t: its column here, or -1
    __shared__ int sh_slice, sh_st, sh_ws, sh_cl;

    const int n = (int)n64, s0 = (int)s064, width = n - s0;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) {
        // block 0 publishes its XCD (or, beside a trailing update that
        // leaves it alone, the XCD is 0); blocks elsewhere leave, the
        // others take slices from a counter in that XCD's L2
        const int x = xcc_id();
        int e = x;
        if (w.state->status != kStatusOk) {
            e = -1;
        } else if (on_xcc0) {
            e = 0;
        } else if (blockIdx.x == 0) {
            st_agent(&w.claim[1], x);
        } else {
            const uint64_t t0 = now_ticks();
            while ((e = ld_agent(&w.claim[1])) < 0) {
                if (now_ticks() - t0 > kWaitTicks) {
                    st_agent(&w.state->status, (int)kStatusAborted);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        sh_slice = (e == x) ? atomicAdd(&w.claim[0], 1) : -1;
    }
    __syncthreads();
    const int slice = sh_slice;
    if (slice < 0 || slice >= nslices) return;

    T* __restrict__ W = w.W;
    const int64_t ldw = w.ldw;
    const int cbase = slice * CP + wv * CPW; // first column of this wave (from s0)
    for (int t = tid; t < CP; t += kSplitThreads) {
        const int col = slice * CP + t;
        const bool ok = col < width;
        cpos[t] = ok ? s0 + col : -1;
        cstep[t] = ok ? kSplitNone : -1; // active at step k: cstep >= k
        cid[t] = ok ? w.perm[s0 + col] : 0x7fffffff;
        prow[0][t] = prow[1][t] = T(0);
        nrow[0][t] = nrow[1][t] = T(0);
    }
    if (slice == 0) {
        // this map set's entries from two panels back return to the
        // identity; the stores complete before the first barrier, so before
        // any record of this block, so before any block's final map entries
        for (int t = tid; t < kMaxPanel; t += kSplitThreads) {
            const int d = w.moved[t];
            if (d >= 0) {
                w.colsrc[d] = d;
                w.moved[t] = -1;
            }
        }
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    }
    for (int t = tid; t < kMaxPanel; t += kSplitThreads) {
        mult[0][t] = mult[1][t] = T(0);
        const int cl = t - slice * CP; // position s0+t holds column t at the start
        invpos[t] = (cl >= 0 && cl < CP && t < width) ? cl : -1;
    }

    // the slice's rows, loaded coalesced and transposed through LDS, TC
    // columns a pass.  One buffer descriptor covers the panel rows (rows
    // past nb read as zero); lane L reads column L % TC of the pass, rows
    // L / TC + RS u (RS rows a load).
    constexpr int RS = kWave / TC;
    const int c_l = lane % TC, r_l = lane / TC;
    const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
        W + (int64_t)s0 * ldw, 0, (int)(sizeof(T) * (int64_t)nb * ldw), 0x00020000);
    const int row_bytes = (int)(sizeof(T) * ldw);
    T x[H][CPW];
    T* tw = tb + wv * 64 * TBLD;
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
        for (int j = 0; j < CPW / TC; ++j) {
            const bool col_ok = cbase + j * TC + c_l < width;
            const int voff = r_l * row_bytes +
                             (int)sizeof(T) * (s0 + (col_ok ? cbase + j * TC + c_l : 0));
            T t[TC];
#pragma unroll
            for (int u = 0; u < TC; ++u) {
                const T v = buf_load<T>(prs, voff, (64 * h + RS * u) * row_bytes);
                t[u] = col_ok ? v : T(0);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < TC; ++u) tw[(r_l + RS * u) * TBLD + c_l] = t[u];
            __syncthreads();
#pragma unroll
            for (int c = 0; c < TC; ++c) x[h][j * TC + c] = tw[lane * TBLD + c];
        }
    }

    const __amdgpu_buffer_rsrc_t stat = l2_rsrc(&w.state->status, sizeof(int));
    // row 0 for the first step's candidate (no step applied yet)
    {
        const int pb0 = (s0 & 1) ^ 1;
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < CPW; ++c) nrow[pb0][wv * CPW + c] = x[0][c];
        }
    }
    __syncthreads();
    // the scan's columns lane + 64 q: their ids, and which are still active
    int cidr[CP / kWave];
    uint32_t act = 0;
#pragma unroll
    for (int q = 0; q < CP / kWave; ++q) {
        cidr[q] = cid[lane + kWave * q];
        if (cstep[lane + kWave * q] == kSplitNone) act |= 1u << q;
    }
    T keep0 = T(0), keep1 = T(0); // wave 0: the last retiring column's multipliers
    int keep_s = -1, keep_k = 0;
    // One step.  B0: step k-1 still reaches rows 0..63; HN: half of row k+1.
    // Returns false once the panel stops (a singular or non-finite pivot
    // row, or an aborted wait).
    auto step = [&](auto b0c, auto hnc, int k) -> bool {
        constexpr bool B0 = decltype(b0c)::value;
        constexpr int HN = decltype(hnc)::value;
        const int s = s0 + k, b = s & 1, pb = b ^ 1;
        // 1. row k (the staged row with step k-1 applied here) and the
        //    block's candidate, reduced by every wave alike
        const T mk = mult[pb][k];
        uint64_t a = 0, key = ~0ull;
        bool bad = false;
#pragma unroll
        for (int q = 0; q < CP / kWave; ++q) {
            const int cl = lane + kWave * q;
            const T v = fma(-mk, prow[pb][cl], nrow[pb][cl]);
            if (wv == 0) prow[b][cl] = v;
            if ((act >> q) & 1u) {
                const double av = fabs((double)v);
                if (!isfinite(av)) {
                    bad = true;
                } else {
                    const uint64_t kk = ((uint64_t)(uint32_t)cidr[q] << 32) |
                                        ((uint64_t)(v < T(0)) << 31) | (uint64_t)cl;
                    split_take(a, key, (uint64_t)__double_as_longlong(av), kk);
                }
            }
        }
        wave_best_fast(a, key);
        bad = __builtin_amdgcn_ballot_w64(bad) != 0;
        const bool has = key != ~0ull;
        const int clw = has ? (int)(key & 0xffffu) : 0;
        // 2. the owning wave posts the column (step k-1 applied here), then
        //    the record
        if (wv == clw / CPW) {
            const int b2 = b * kSplitSlices + slice;
            if (has) {
                // the column by a register index that every lane shares,
                // within a vector of at most 32 registers (the largest such
                // an index reaches without going through memory)
                constexpr int NV = CPW < 128 / (int)sizeof(T) ? CPW : 128 / (int)sizeof(T);
                typedef T xvec __attribute__((ext_vector_type(NV)));
                const int cw = __builtin_amdgcn_readfirstlane(clw % CPW);
                const int cq = cw / NV, ce = cw % NV;
                T y0 = T(0), y1 = T(0); // rows 0..63 matter only while k < 63
#pragma unroll
                for (int q = 0; q < CPW / NV; ++q) {
                    if (q == cq) {
                        xvec v0, v1;
#pragma unroll
                        for (int e = 0; e < NV; ++e) {
                            v0[e] = x[0][q * NV + e];
                            v1[e] = x[H - 1][q * NV + e];
                        }
                        if (B0) y0 = v0[ce];
                        if (H > 1) y1 = v1[ce];
                    }
                }
                const T r = prow[pb][clw];
                y0 = fma(-mult[pb][lane], r, y0);
                T* col = w.xcol + (size_t)b2 * kMaxPanel;
                col[lane] = y0;
                if (H > 1) {
                    y1 = fma(-mult[pb][64 + lane], r, y1);
                    col[64 + lane] = y1;
                }
                __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            }
            if (lane == 0) {
                const uint64_t pos = has ? (uint64_t)(cpos[clw] & 0xffffff) : 0;
                const uint64_t id = has ? ((key >> 32) & 0xffffff) : 0;
                const uint64_t w0 = a | ((uint64_t)((s >> 1) & 1) << 63);
                const uint64_t w1 = ((uint64_t)((s + 1) & 0x3fff) << 50) |
                                    (((key >> 31) & 1ull) << 49) |
                                    ((uint64_t)bad << 48) | (id << 24) | pos;
                typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
                *reinterpret_cast<u64x2*>(w.xrec + 2 * b2) = u64x2{w0, w1};
            }
        }
        // 3. step k-1 on the registers (a retired column is updated too:
        //    only its rows up to its own step are kept, and its multipliers
        //    went to W when it retired)
        {
            const T m0 = -mult[pb][lane], m1 = -mult[pb][64 + lane];
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                // the pivot row's entry is the same in every lane: keep it
                // in scalar registers
                const T r = wave_uniform(prow[pb][wv * CPW + c]);
                if (B0) x[0][c] = fma(m0, r, x[0][c]);
                if (H > 1) x[H - 1][c] = fma(m1, r, x[H - 1][c]);
            }
            // a use of the updated data here, so that the update stays
            // before the barrier below rather than being moved onto the
            // next step's critical path
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                if (B0) asm volatile("" ::"v"(x[0][c]));
                if (H > 1) asm volatile("" ::"v"(x[H - 1][c]));
            }
        }
        // 4. row k+1 (step k-1 now applied) staged for the next step's
        //    candidate by the lane holding it
        if (lane == ((k + 1) & 63)) {
#pragma unroll
            for (int c = 0; c < CPW; ++c) nrow[b][wv * CPW + c] = x[HN < H ? HN : 0][c];
        }
        // 5. wave 0 takes the winner
        if (wv == 0) {
            const __amdgpu_buffer_rsrc_t rec =
                l2_rsrc(w.xrec + 2 * b * kSplitSlices, 16 * kSplitSlices);
            const uint64_t gbit = (uint64_t)((s >> 1) & 1);
            const uint64_t tag = (uint64_t)((s + 1) & 0x3fff);
            uint64_t r0 = 0, r1 = 0;
            int stw = kStatusOk;
            long spins = 0;
            const uint64_t t0 = now_ticks();
            for (;;) {
                bool ok = true;
                if (lane < nslices) {
                    asm volatile("" ::: "memory");
                    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rec, lane * 16, 0,
                                                                         kL2Policy);
                    r0 = ((uint64_t)(uint32_t)v[1] << 32) | (uint32_t)v[0];
                    r1 = ((uint64_t)(uint32_t)v[3] << 32) | (uint32_t)v[2];
                    ok = (r0 >> 63) == gbit && (r1 >> 50) == tag;
                }
                if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
                ++spins;
                if ((spins & 63) == 0) {
                    if (now_ticks() - t0 > kWaitTicks) {
                        stw = kStatusAborted;
                        break;
                    }
                    if (__builtin_amdgcn_readfirstlane(l2_poll(stat, 0)) != kStatusOk) {
                        stw = kStatusAborted; // another block stopped the panel
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (stw == kStatusOk) {
                const bool in = lane < nslices;
                uint64_t ga = in ? (r0 & 0x7fffffffffffffffull) : 0ull;
                uint64_t gk = in ? ((((r1 >> 24) & 0xffffff) << 32) | (uint64_t)lane) : ~0ull;
                const bool gbad = __builtin_amdgcn_ballot_w64(in && ((r1 >> 48) & 1)) != 0;
                wave_best_fast(ga, gk);
                const int ws = (int)(gk & 0xff);
                const uint64_t wr1 = readlane64(r1, ws);
                if (gbad)
                    stw = kStatusNonfinite;
                else if (ga == 0 || gk == ~0ull)
                    stw = kStatusSingular;
                if (stw == kStatusOk) {
                    const double mag = __longlong_as_double((long long)ga);
                    const double p = ((wr1 >> 49) & 1) ? -mag : mag;
                    const int l = (int)(wr1 & 0xffffff);
                    const T pt = (T)p;
                    const __amdgpu_buffer_rsrc_t cr = l2_rsrc(
                        w.xcol + (size_t)(b * kSplitSlices + ws) * kMaxPanel,
                        sizeof(T) * kMaxPanel);
                    // the column's loads first; the reciprocal of the pivot
                    // and the bookkeeping below overlap them
                    const T c0 = l2_load<T>(cr, lane);
                    const T c1 = H > 1 ? l2_load<T>(cr, 64 + lane) : T(0);
                    const T rp = T(1) / pt;
                    if (lane == 0) {
                        pv[k] = p;
                        pl[k] = l;
                        if (ws == slice) {
                            cstep[clw] = k;
                            w.srcp[k] = s0 + slice * CP + clw; // where it started
                        }
                        sh_ws = ws;
                        sh_cl = clw;
                        // the exchange: the column at position s moves to l,
                        // the pivot column to s (positions past the panel
                        // are never looked up, so only theirs is not kept)
                        if (l != s) {
                            const int jt = invpos[k]; // the column at s, if here
                            if (ws == slice) cpos[clw] = s;
                            if (jt >= 0) cpos[jt] = l;
                            invpos[k] = (ws == slice) ? clw : -1;
                            if (l - s0 < nb) invpos[l - s0] = jt;
                        }
                    }
                    const bool in0 = lane > k && lane < nb;
                    const bool in1 = 64 + lane > k && 64 + lane < nb;
                    mult[b][lane] = in0 ? c0 * rp : T(0);
                    mult[b][64 + lane] = in1 ? c1 * rp : T(0);
                    if (ws == slice) { // stored after the barrier
                        keep0 = in0 ? c0 : T(0);
                        keep1 = in1 ? c1 : T(0);
                        keep_s = s;
                        keep_k = k;
                    }
                }
            }
            if (lane == 0) sh_st = stw;
        }
        __syncthreads();
        const int st = sh_st;
        if (st == kStatusOk && sh_ws == slice && lane == (sh_cl & 63))
            act &= ~(1u << (sh_cl >> 6)); // the column this step retired
        if (wv == 0 && keep_s >= 0) {
            // the retiring column's multipliers, at the position the column
            // takes (s), for the rows below its step
            if (lane > keep_k && lane < nb)
                buf_store<T>(keep0, prs, lane * row_bytes + (int)sizeof(T) * keep_s, 0);
            if (64 + lane > keep_k && 64 + lane < nb)
                buf_store<T>(keep1, prs, (64 + lane) * row_bytes + (int)sizeof(T) * keep_s, 0);
            keep_s = -1;
        }
        if (st == kStatusOk) return true;
        if (slice == 0) { // the steps taken so far, then the failed one
            for (int t = tid; t < k; t += kSplitThreads) {
                w.piv_pos[s0 + t] = pl[t];
                w.piv_val[s0 + t] = pv[t];
            }
            if (tid == 0) {
                w.piv_pos[s] = -1;
                w.piv_val[s] = 0.0;
                st_agent(&w.state->bad_step, s);
                st_agent(&w.state->status, st);
            }
        } else if (tid == 0 && st == kStatusAborted) {
            st_agent(&w.state->status, st);
        }
        return false;
    };
    using B_on = std::true_type;
    using B_off = std::false_type;
    using H0 = std::integral_constant<int, 0>;
    using H1 = std::integral_constant<int, 1>;
    const int nbA = H > 1 ? (nb < 63 ? nb : 63) : nb;
    // one exit after the loops: a return from inside them would leave the
    // data without a use on that path, and the register allocator then
    // keeps two copies of it alive through every step
    bool live = true;
#pragma unroll 1
    for (int k = 0; k < nbA && live; ++k)
        live = step(B_on{}, H0{}, k);
    if (H > 1) {
        if (live && nb > 63) live = step(B_on{}, H1{}, 63);
#pragma unroll 1
        for (int k = 64; k < nb && live; ++k)
            live = step(B_off{}, H1{}, k);
    }
    if (!live) return;

    // the factored rows at the columns' final positions (rows past nb fall
    // outside the descriptor and are dropped; columns past the panel's
    // width have cstep -1 and are skipped).  The lane index goes through an
    // empty asm so that the addresses below are formed here rather than kept
    // in registers from the loads across the whole step loop.
    int lane_f = lane;
    asm volatile("" : "+v"(lane_f));
    const int cf_l = lane_f % TC, rf_l = lane_f / TC;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int i = 64 * h + lane_f;
        const T p = (T)pv[i < nb ? i : 0];
#pragma unroll
        for (int j = 0; j < CPW / TC; ++j) {
            __syncthreads();
#pragma unroll
            for (int c = 0; c < TC; ++c) {
                if (c % 4 == 0) __builtin_amdgcn_sched_barrier(0); // a few divisions at a time
                const T v = x[h][j * TC + c];
                tw[lane_f * TBLD + c] = (i < cstep[wv * CPW + j * TC + c]) ? v / p : v;
            }
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();
            // rows below a retired column's step hold its multipliers already
            const int colj = wv * CPW + j * TC + cf_l;
            const int pos_l = cpos[colj];
            const int soff = rf_l * row_bytes +
                             (int)sizeof(T) * (cbase + j * TC + cf_l < width ? pos_l : s0);
            const int cs_l = cstep[colj];
#pragma unroll
            for (int u = 0; u < TC; ++u) {
                const int r = 64 * h + rf_l + RS * u;
                if (r <= cs_l)
                    buf_store<T>(tw[(rf_l + RS * u) * TBLD + cf_l], prs, soff,
                                 (64 * h + RS * u) * row_bytes);
            }
        }
    }
    for (int t = tid; t < CP; t += kSplitThreads)
        if (slice * CP + t < width) w.perm[cpos[t]] = cid[t];
    // the column maps of the panel's exchanges for the rows below it (w
    // carries this panel's set): a trailing position d >= pend that a step
    // exchanged reads from where its final column started (srcp, the panel
    // columns' sources, went out as the steps were taken)
    for (int t = tid; t < CP; t += kSplitThreads) {
        const int col = slice * CP + t, d = cpos[t];
        if (col < width && d >= s0 + nb && d != s0 + col) w.colsrc[d] = s0 + col;
    }
    if (slice == 0)
        for (int t = tid; t < nb; t += kSplitThreads) {
            w.piv_pos[s0 + t] = pl[t];
            w.piv_val[s0 + t] = pv[t];
            if (pl[t] >= s0 + nb) w.moved[t] = pl[t];
        }
}


// Panel rows published before the last steps: apply the exchanges of the
// steps after their own (one wavefront per row; sources found by undoing
// the exchanges in reverse, every value read before any is written).
template <typename T>
__device__ void panel_row_fixup(BlkWork<T>& w, int64_t s0, int nb, int64_t u,
                                const int* lp)
{
    const int lane = threadIdx.x & 63;
    const int rel = (int)(u - s0);
    T* row = w.W + u * w.ldw;
    const int lp0 = lane < nb ? lp[lane] : 0;
    const int lp1 = lane + kWave < nb ? lp[lane + kWave] : 0;
    int d[4], pos[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + q * kWave; // 0..255: steps u+1.. and their l
        const int t = rel + 1 + (e >> 1);
        d[q] = t < nb ? ((e & 1) ? lp[t] : (int)s0 + t) : -1;
        pos[q] = d[q];
    }
    undo_exchanges<4>(pos, (int)s0, rel + 1, nb, lp0, lp1);
    T val[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (d[q] >= 0 && pos[q] != d[q]) val[q] = row[pos[q]];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (d[q] >= 0 && pos[q] != d[q]) row[d[q]] = val[q];
}

// Elements per thread for a row of `width` active entries, or 0 when the
// row is wider than the register-resident kernels handle.
static int step_ept(int64_t width)
{
    for (int e = 1; e <= 16; e *= 2)
        if (width <= (int64_t)e * kStepThreads) return e;
    return 0;
}

// Launch the single-XCD panel over rows s0+1 .. pend-1 (NT threads, EPT
// entries each): R rows per slot, at most 32 slots (one per compute unit of
// an XCD).  The panel's widths are all within the register-resident head
// kernel's, which writes the column-id snapshot the panel starts from.
template <typename T, int NT, int EPT>
static void launch_panel_x(int64_t n, int64_t s0, int64_t pend,
                           const BlkWork<T>& w, hipStream_t stream)
{
    const int rows = (int)(pend - 1 - s0);
    const int R = (rows + 31) / 32; // 1 .. 4 (rows <= 127)
    const int nslots = (rows + R - 1) / R; // slot q: rows s0+1+qR ..
    const dim3 grid((unsigned)(8 * nslots)), block(NT);
    if (R == 1)
        hipLaunchKernelGGL((blk_panel_x<T, NT, EPT, 1>), grid, block, 0, stream, n, s0, pend, nslots, w);
    else if (R == 2)
        hipLaunchKernelGGL((blk_panel_x<T, NT, EPT, 2>), grid, block, 0, stream, n, s0, pend, nslots, w);
    else if (R == 3)
        hipLaunchKernelGGL((blk_panel_x<T, NT, EPT, 3>), grid, block, 0, stream, n, s0, pend, nslots, w);
    else
        hipLaunchKernelGGL((blk_panel_x<T, NT, EPT, 4>), grid, block, 0, stream, n, s0, pend, nslots, w);
}

static bool panel_x_fits(int64_t width) { return width <= 768 * 11; }

// Single-XCD panel for a row width; false when wider than it handles
// (4 rows of up to 11 entries per thread keep every slot's rows in
// registers).
template <typename T>
static bool try_panel_x(int64_t n, int64_t s0, int64_t pend,
                        const BlkWork<T>& w, hipStream_t stream)
{
    const int64_t width = n - s0;
    if (width <= 512) launch_panel_x<T, 512, 1>(n, s0, pend, w, stream);
    else if (width <= 1024) launch_panel_x<T, 512, 2>(n, s0, pend, w, stream);
    else if (width <= 2048) launch_panel_x<T, 512, 4>(n, s0, pend, w, stream);
    else if (width <= 4096) launch_panel_x<T, 512, 8>(n, s0, pend, w, stream);
    else if (panel_x_fits(width)) launch_panel_x<T, 768, 11>(n, s0, pend, w, stream);
    else return false;
    return true;
}

template <typename T, int CPW, int H = 2>
static hipError_t launch_split(int64_t n, int64_t s0, int nb, const BlkWork<T>& w,
                               hipStream_t stream, bool on_xcc0)
{
    static bool attr_set = false; // guarded by g_sched_mu (held by the caller)
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&blk_panel_split<T, CPW, H>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)split_lds_bytes<T, CPW>());
        if (e != hipSuccess) return note_hip_error(e);
        attr_set = true;
    }
    constexpr int CP = kSplitWaves * CPW;
    const int slices = (int)((n - s0 + CP - 1) / CP);
    const size_t lds = split_lds_bytes<T, CPW>();
    hipLaunchKernelGGL((blk_panel_split<T, CPW, H>), dim3((unsigned)(8 * slices)),
                       dim3(kSplitThreads), lds, stream, n, s0, nb, slices,
                       on_xcc0 ? 1 : 0, w);
    return hipSuccess;
}

// Most columns per wavefront of the column-split panel for a panel of nb
// rows: each lane holds ceil(nb / 64) x CPW values in registers, at most
// 128 of them -- 64 columns for FP32, or for FP64 panels of at most 64 rows,
// else 32 -- so one XCD's slices span up to 16384 columns (8192 for FP64
// panels of more than 64 rows).
template <typename T>
constexpr int split_cpw_max(int nb)
{
    return (sizeof(T) == 4 || nb <= 64) ? 64 : 32;
}

// `on`: the column-split setting, read once per call; `beside`: the panel
// runs beside a trailing update and keeps one compute unit of its XCD free.
template <typename T>
static bool split_fits(int64_t width, int nb, bool on, bool beside = false)
{
    const int64_t slices = beside ? kSplitSlices - 1 : kSplitSlices;
    return on && width <= slices * kSplitWaves * split_cpw_max<T>(nb);
}

// The column-split panel for a panel of width n - s0 (split_fits): the
// fewest columns per wave that keep the slices within 32.  Beside a
// trailing update (on_xcc0: the update leaves XCD 0 to the panel) at most
// 31 where the width allows, so that one compute unit there stays free for
// that update's blocks that land on it and leave: with every unit held,
// its blocks on the other XCDs would wait on them (workgroups are
// dispatched in order).
template <typename T>
static hipError_t launch_panel_split(int64_t n, int64_t s0, int nb,
                                     const BlkWork<T>& w, hipStream_t stream,
                                     bool on_xcc0)
{
    const int64_t width = n - s0, slices = on_xcc0 ? kSplitSlices - 1 : kSplitSlices;
    if (width <= slices * kSplitWaves * 8)
        return launch_split<T, 8>(n, s0, nb, w, stream, on_xcc0);
    if (width <= slices * kSplitWaves * 16)
        return launch_split<T, 16>(n, s0, nb, w, stream, on_xcc0);
    if (width <= slices * kSplitWaves * 32)
        return launch_split<T, 32>(n, s0, nb, w, stream, on_xcc0);
    // wider (split_fits): 64 columns per wavefront, the panel's 128 rows in
    // FP32, at most 64 rows in FP64
    if constexpr (sizeof(T) == 4)
        return launch_split<T, 64, 2>(n, s0, nb, w, stream, on_xcc0);
    else
        return launch_split<T, 64, 1>(n, s0, nb, w, stream, on_xcc0);
}

template <typename T>
static void launch_head(int64_t n, int64_t s, const BlkWork<T>& w,
                        hipStream_t stream)
{
    switch (step_ept(n - s)) {
#define MC_HEAD(E)                                                            \
    case E:                                                                   \
        hipLaunchKernelGGL((blk_head_r<T, E>), dim3(1), dim3(kStepThreads),  \
                           0, stream, n, s, w);                               \
        return;
        MC_HEAD(1) MC_HEAD(2) MC_HEAD(4) MC_HEAD(8) MC_HEAD(16)
#undef MC_HEAD
    default:
        hipLaunchKernelGGL(blk_head<T>, dim3(1), dim3(kBlkThreads), 0, stream,
                           n, s, w);
    }
}

template <typename T>
static void launch_step(int64_t n, int64_t s, int64_t s0, int64_t pend,
                        const BlkWork<T>& w, hipStream_t stream)
{
    const int64_t blocks = std::max<int64_t>(1, pend - 1 - s);
    switch (step_ept(n - s - 1)) {
#define MC_STEP(E)                                                            \
    case E:                                                                   \
        hipLaunchKernelGGL((blk_step_r<T, E>), dim3((unsigned)blocks),       \
                           dim3(kStepThreads), 0, stream, n, s, s0, pend, w); \
        return;
        MC_STEP(1) MC_STEP(2) MC_STEP(4) MC_STEP(8) MC_STEP(16)
#undef MC_STEP
    default:
        hipLaunchKernelGGL(blk_step<T>, dim3((unsigned)blocks),
                           dim3(kBlkThreads), 0, stream, n, s, s0, pend, w);
    }
}

// For the rows below the panel, where did each moved column come from?
// Position s0+t exchanged contents with position l_t at step s0+t, so the
// source of a destination is found by undoing the exchanges in reverse.
// The same block also inverts the 16 x 16 diagonal blocks of the unit upper
// triangle U11 of the factored panel (back substitution, one column per
// thread), for the triangular solve below.
template <typename T>
__device__ void panel_row_fixup(BlkWork<T>& w, int64_t s0, int nb, int64_t u,
                                const int* lp);


// Fix-up of the panel rows published by the persistent panel kernel (four
// rows per block).  Runs before blk_perm, which reads the fixed rows (U11).
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_fixup(int64_t s0, int nb, BlkWork<T> w)
{
    __shared__ int lp[kMaxPanel];
    if (w.state->status != kStatusOk) return;
    for (int t = threadIdx.x; t < nb; t += kBlkThreads) lp[t] = w.piv_pos[s0 + t];
    __syncthreads();
    const int64_t u = s0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u < s0 + nb - 1) panel_row_fixup(w, s0, nb, u, lp);
}

// Fix-up after the single-XCD panel, one block per panel row u: rows after
// the first were published unfactored, so factor them in place (row u of
// Section 2.3 divided by its pivot, whose slot takes the entry at u; the
// multipliers left of u stay), then apply the later steps' exchanges.
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_fixup_x(int64_t n, int64_t s0, int nb, BlkWork<T> w)
{
    __shared__ int lp[kMaxPanel];
    if (w.state->status != kStatusOk) return;
    for (int t = threadIdx.x; t < nb; t += kBlkThreads) lp[t] = w.piv_pos[s0 + t];
    const int64_t u = s0 + blockIdx.x;
    if (u > s0) {
        T* row = w.W + u * w.ldw;
        const T p = (T)w.piv_val[u];
        const int64_t l = w.piv_pos[u];
        const T vu = row[u];
        __syncthreads(); // every thread has vu before position u is written
        constexpr int U8 = 16; // entries per thread per pass, all loads first
        for (int64_t j0 = u + threadIdx.x; j0 < n; j0 += (int64_t)U8 * kBlkThreads) {
            T x[U8];
#pragma unroll
            for (int q = 0; q < U8; ++q) {
                const int64_t j = j0 + (int64_t)q * kBlkThreads;
                x[q] = j < n ? row[j] : T(0);
            }
#pragma unroll
            for (int q = 0; q < U8; ++q) {
                const int64_t j = j0 + (int64_t)q * kBlkThreads;
                if (j < n) row[j] = (j == u) ? p : ((j == l) ? vu : x[q]) / p;
            }
        }
    }
    __syncthreads(); // the factored row (and lp) is visible to the block
    if (u < s0 + nb - 1 && threadIdx.x < kWave) panel_row_fixup(w, s0, nb, u, lp);
}

template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_perm(int64_t s0, int nb, BlkWork<T> w)
{
    __shared__ int lp[kMaxPanel];
    if (w.state->status != kStatusOk) return;
    const int tid = threadIdx.x;
    if (tid == 0) { // the next panel's blocks elect an XCD afresh; the
        w.claim[0] = 0; // trailing update's tile counter starts at zero
        w.claim[1] = -1;
        w.claim[2] = 0;
    }
    for (int t = tid; t < kMaxPanel; t += kBlkThreads) {
        const int d = w.moved[t];
        if (d >= 0) {
            w.colsrc[d] = d;
            w.moved[t] = -1;
        }
    }
    for (int t = tid; t < nb; t += kBlkThreads) lp[t] = w.piv_pos[s0 + t];
    __syncthreads();
    const int64_t pend = s0 + nb;
    static_assert(kMaxPanel <= 2 * kWave, "partners held in two registers");
    {
        const int lane = tid & (kWave - 1);
        const int lp0 = lane < nb ? lp[lane] : 0;
        const int lp1 = lane + kWave < nb ? lp[lane + kWave] : 0;
        // destinations s0+t and lp[t], traced together; every lane runs the
        // trace (readlane reads lanes that a branch would switch off)
        const int t = tid < nb ? tid : 0;
        const int d = lp[t];
        int pos[2] = {(int)s0 + t, d};
        undo_exchanges<2>(pos, (int)s0, 0, nb, lp0, lp1);
        if (tid < nb) {
            w.srcp[tid] = pos[0];
            if (d >= pend) {
                w.colsrc[d] = pos[1];
                w.moved[tid] = d;
            }
        }
    }
    // diagonal-block inverses: column c of block J solves U_JJ x = e_c,
    // with the blocks staged in LDS first (one coalesced read)
    const int nblk = (nb + 15) / 16;
    const T* U = w.W + s0 * w.ldw + s0;
    __shared__ T Ud[kMaxPanel / 16][16][17];
    for (int e = tid; e < nblk * 256; e += kBlkThreads) {
        const int J = e >> 8, r = (e >> 4) & 15, v = e & 15;
        const int pr = 16 * J + r, pv = 16 * J + v;
        Ud[J][r][v] = (pv < nb && pr < nb) ? U[(int64_t)pr * w.ldw + pv] : T(0);
    }
    __syncthreads();
    for (int e = tid; e < nblk * 16; e += kBlkThreads) {
        const int J = e >> 4, c = e & 15;
        T x[16]; // column form, as in the solve's own inverses
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = (r == c) ? T(1) : T(0);
#pragma unroll
        for (int v = 15; v >= 1; --v) {
            if (v > c) continue;
#pragma unroll
            for (int r = 0; r < v; ++r) x[r] = fma(-Ud[J][r][v], x[v], x[r]);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) w.dinv[(J * 16 + r) * 16 + c] = x[r];
    }
}

// L21 = A21 * U11^{-1} on the matrix cores, one wavefront per 16 rows, as
// its transpose X^T = U11^{-T} A21^T in 16-row blocks J of X^T (forward
// substitution by blocks):
//     R_J = A21^T[J, :] - sum_{K<J} U11[K, J]^T X^T[K, :]   (MFMA, K = 16 per block)
//     X^T[J, :] = inv(U11[J, J])^T R_J                      (MFMA)
// with A21[i][t] = W[i][srcp[t]] (the exchanges folded into the load).  In
// this form a finished block, in the accumulator layout, is already the
// second operand of the later blocks' products: the rows of X^T a lane
// holds are the k values it supplies, so X never leaves the registers.
// Rows past n and columns past nb are zeros.
// Only the first `aw` wavefronts of a block take rows (16 each): the gather
// reads one cache line per entry, and one compute unit keeps only so many
// lines in flight, so a launch spreads its rows over as many compute units
// as it can (all four wavefronts still stage U11 and form the inverses).
template <typename T, bool INV>
__global__ void __launch_bounds__(kBlkThreads)
blk_trsm_mfma(int64_t n, int64_t s0, int nb, int aw, BlkWork<T> w)
{
    using P = typename MfmaFor<T>::P;
    extern __shared__ unsigned char smem_raw[];
    const int nblk = (nb + 15) / 16;
    if (w.state->status != kStatusOk) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    __shared__ int src_sh[kMaxPanel];
    const int64_t pend = s0 + nb;
    const int64_t i0 = pend + (int64_t)blockIdx.x * (16 * aw) + wid * 16;
    const bool rows_here = wid < aw;
    const T* __restrict__ W = w.W;
    const int64_t ldw = w.ldw;
    const T* U = W + s0 * ldw + s0;
    const int cin = lane & 15;
    // U11's strictly upper 16x16 blocks (K < J at tri(K, J) = J(J-1)/2 + K)
    // and the inverted diagonal blocks, both in LDS: the solve's chain then
    // waits on no global load.
    constexpr int kMaxBlk = kMaxPanel / 16;
    constexpr int kMaxTri = kMaxBlk * (kMaxBlk - 1) / 2;
    static_assert(kBlkThreads == 256, "one 16x16 block element per thread");
    const int ntri = nblk * (nblk - 1) / 2;
    T* Ub = reinterpret_cast<T*>(smem_raw) + kMaxBlk * 272; // after the staging
    T* Dv = Ub + ntri * 256;
    for (int t = tid; t < nb; t += kBlkThreads) src_sh[t] = w.srcp[t];
    if (INV && blockIdx.x == 0 && tid == 0) { // after a column-split panel:
        w.claim[0] = 0;                       // the next panel's blocks
        w.claim[1] = -1;                      // elect an XCD afresh; the
        w.claim[2] = 0;                       // update's tile counter
    }
    {
        const int er = tid >> 4, ec = tid & 15;
        T st[kMaxTri + kMaxBlk];
        int bi = 0;
#pragma unroll
        for (int J = 1; J < kMaxBlk; ++J)
#pragma unroll
            for (int K = 0; K < J; ++K, ++bi) {
                const int t = 16 * J + ec;
                st[bi] = (J < nblk && t < nb) ? U[(int64_t)(16 * K + er) * ldw + t] : T(0);
            }
#pragma unroll
        for (int J = 0; J < kMaxBlk; ++J) {
            // the inverted diagonal blocks, or (INV) the blocks themselves
            const int t = 16 * J + ec;
            if (INV)
                st[kMaxTri + J] = (J < nblk && t < nb) ? U[(int64_t)(16 * J + er) * ldw + t] : T(0);
            else
                st[kMaxTri + J] = J < nblk ? w.dinv[J * 256 + tid] : T(0);
        }
        bi = 0;
#pragma unroll
        for (int J = 1; J < kMaxBlk; ++J)
#pragma unroll
            for (int K = 0; K < J; ++K, ++bi)
                if (J < nblk) Ub[bi * 256 + tid] = st[bi];
#pragma unroll
        for (int J = 0; J < kMaxBlk; ++J)
            if (J < nblk) {
                if (INV) // the blocks, padded, for the inverses below
                    reinterpret_cast<T*>(smem_raw)[J * 272 + er * 17 + ec] = st[kMaxTri + J];
                else
                    Dv[J * 256 + tid] = st[kMaxTri + J];
            }
    }
    __syncthreads();
    // every gathered entry of A21 first (one memory latency for all
    // blocks): lane (cin, r) of block J takes row i0 + cin, column
    // 16 J + P::drow(lane, r), in the accumulator layout of X^T
    T g[kMaxBlk][4];
    const int64_t grow = i0 + cin;
#pragma unroll
    for (int J = 0; J < kMaxBlk; ++J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = 16 * J + P::drow(lane, r);
            g[J][r] = (rows_here && J < nblk && grow < n && t < nb)
                          ? W[grow * ldw + src_sh[t]]
                          : T(0);
        }
    }
    if (INV) {
        // the diagonal blocks' inverses (unit upper triangular: column c of
        // block J solves U_JJ x = e_c by back substitution), while the
        // gathers above are in flight
        const T* Ud = reinterpret_cast<const T*>(smem_raw);
        if (tid < nblk * 16) {
            const int J = tid >> 4, c = tid & 15;
            // column form: once x[v] is final, every row above takes its
            // share at once (a dependency chain of 15 FMAs, not ~120)
            T x[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) x[r] = (r == c) ? T(1) : T(0);
#pragma unroll
            for (int v = 15; v >= 1; --v) {
                if (v > c) continue; // x[v] = 0 there
#pragma unroll
                for (int r = 0; r < v; ++r) x[r] = fma(-Ud[J * 272 + r * 17 + v], x[v], x[r]);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) Dv[(J * 16 + r) * 16 + c] = x[r];
        }
        __syncthreads(); // the inverses are in
    }
    if (!rows_here) return;
    typename P::Acc xt[kMaxBlk]; // finished blocks of X^T
#pragma unroll
    for (int J = 0; J < kMaxBlk; ++J) {
        if (J >= nblk) break;
        typename P::Acc acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = g[J][r];
#pragma unroll
        for (int K = 0; K < kMaxBlk; ++K) {
            if (K >= J) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // k = P::drow(lane, q): row k of block K of X^T is this
                // lane's register q; A supplies U11[16 K + k][16 J + cin]
                const T a = -Ub[(J * (J - 1) / 2 + K) * 256 + P::drow(lane, q) * 16 + cin];
                acc = P::mma(a, xt[K][q], acc);
            }
        }
        typename P::Acc x = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q) // inv(U_JJ)[k][cin] against row k of R_J
            x = P::mma(Dv[(J * 16 + P::drow(lane, q)) * 16 + cin], acc[q], x);
        xt[J] = x;
    }
    // L21[i0 + cin][16 J + P::drow(lane, r)] = X^T[...][cin]
    if (grow < n) {
        T* lrow = w.L + (grow - pend) * w.ldl;
#pragma unroll
        for (int J = 0; J < kMaxBlk; ++J) {
            if (J >= nblk) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = 16 * J + P::drow(lane, r);
                if (t < nb) lrow[t] = xt[J][r];
            }
        }
    }
}

// Factor mode (mc_logdet_factor): after a panel's trailing update, put the
// rows' multipliers into their places (positions s0..pend-1 of the rows
// below the panel) ...
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_store_l(int64_t n, int64_t s0, int nb, BlkWork<T> w)
{
    if (w.state->status != kStatusOk) return;
    const int64_t pend = s0 + nb;
    for (int64_t e = blockIdx.x * (int64_t)kBlkThreads + threadIdx.x;
         e < (n - pend) * nb; e += (int64_t)gridDim.x * kBlkThreads) {
        const int64_t i = e / nb, t = e - i * nb;
        w.W[(pend + i) * w.ldw + s0 + t] = w.L[i * w.ldl + t];
    }
}

// ... and apply the panel's column exchanges to the rows above it (their
// entries right of s0 are factored-row entries in the pre-panel order).
// One wavefront per row: every moved value is read before any is written.
template <typename T>
__global__ void __launch_bounds__(kBlkThreads)
blk_swaps_above(int64_t s0, int nb, BlkWork<T> w)
{
    if (w.state->status != kStatusOk) return;
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * (kBlkThreads / kWave) + (threadIdx.x >> 6);
    if (u >= s0) return;
    T* row = w.W + u * w.ldw;
    // destinations: s0+t (t < nb) from srcp[t]; moved[t] from colsrc[moved[t]]
    T v[4];
    int64_t d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + q * kWave; // 0 .. 255
        d[q] = -1;
        if (e < nb) {
            d[q] = s0 + e;
            v[q] = row[w.srcp[e]];
        } else if (e >= kMaxPanel && e - kMaxPanel < nb) {
            const int t = e - kMaxPanel;
            const int64_t dm = w.moved[t];
            if (dm >= 0) {
                d[q] = dm;
                v[q] = row[w.colsrc[dm]];
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (d[q] >= 0) row[d[q]] = v[q];
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
                             : (st == kStatusAborted ? (int64_t)MC_INFO_ABORTED
                                                     : (int64_t)MC_INFO_NONFINITE);
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
static size_t trsm_mfma_lds_bytes(int nb)
{
    const int nblk = (nb + 15) / 16;
    const int ntri = nblk * (nblk - 1) / 2; // strictly upper 16x16 blocks of U11
    // the diagonal blocks' staging (8 of 16 x 17), then U11's strictly upper
    // blocks and the inverted diagonal blocks
    return sizeof(T) * ((size_t)(kMaxPanel / 16) * 272 + (size_t)(ntri + nblk) * 256);
}

// ---- per-device scheduling: one-panel lookahead, and calls one at a time ----
//
// The next panel only needs its own rows brought up to date, so the
// trailing update is split: the next panel's rows on the caller's stream,
// the rest on a second stream, where it runs beside the next panel's
// factorisation.  That panel's chain holds XCD 0 (a column-split panel
// elects it when told to) and the update leaves XCD 0 alone, so neither
// waits for the other's compute units.  Fork and join are events; the
// caller's stream waits for the join before the next triangular solve and
// before returning.  One side stream and event pair per device, reused
// under a lock held while a call enqueues its work.
//
// A column-split panel needs all of its slices resident together on one
// XCD.  Two blocked calls running at once on one device (from different
// streams) would contend for those compute units, so the device's blocked
// calls run one after another on the GPU: each call's first kernel waits
// for an event the previous call recorded after its last kernel.  Calls
// enqueued under graph capture neither wait nor record (the graph is not
// executed then); replaying such a graph beside another blocked call on the
// same device is the caller's to order.
struct DevSched {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t done = nullptr; // after the device's last blocked call
    bool done_recorded = false;
    bool ready = false, failed = false;
    bool all_xccs = false; // the device exposes its eight XCDs (ids 0..7)
};

constexpr int kMaxDevices = 64;
static DevSched g_sched[kMaxDevices];
static std::mutex g_sched_mu; // guards g_sched and every enqueue of a blocked call

// The current device's scheduling state, created on first use; nullptr
// when it cannot be created.  Caller holds g_sched_mu.
static DevSched* sched_get()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    DevSched& d = g_sched[dev];
    if (!d.ready && !d.failed) {
        if (hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&d.join, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&d.done, hipEventDisableTiming) != hipSuccess) {
            d.failed = true;
            (void)hipGetLastError();
            return nullptr;
        }
        int xccs = 0;
        d.all_xccs = hipDeviceGetAttribute(&xccs, hipDeviceAttributeNumberOfXccs, dev) ==
                         hipSuccess && xccs == 8;
        (void)hipGetLastError();
        d.ready = true;
    }
    return d.ready ? &d : nullptr;
}

// The panel-k view of the workspace: alternate column-map sets.
template <typename T>
static BlkWork<T> panel_view(const BlkWork<T>& w, int64_t k)
{
    BlkWork<T> v = w;
    if (k & 1) {
        v.colsrc = w.colsrc_b;
        v.srcp = w.srcp_b;
        v.moved = w.moved_b;
    }
    return v;
}

template <typename T>
static hipError_t trailing(const BlkWork<T>& w, int update, int64_t s0, int nb,
                           int64_t r0, int64_t m, int64_t n, hipStream_t st,
                           unsigned int* tile_ctr)
{
    const int64_t pend = s0 + nb;
    GemmArgs<T> g;
    g.C = w.W;
    g.ldc = w.ldw;
    g.r0 = r0;
    g.c0 = pend;
    g.M = m;
    g.N = n - pend;
    g.K = nb;
    g.L = w.L + (r0 - pend) * w.ldl;
    g.ldl = w.ldl;
    g.U = w.W + s0 * w.ldw;
    g.ldu = w.ldw;
    g.colsrc = w.colsrc;
    g.state = w.state;
    g.tile_ctr = tile_ctr;
    const ProfMark pm = prof_begin(st);
    const hipError_t e = launch_trailing_update(g, update, st);
    if (e != hipSuccess) return e;
    const double flops = 2.0 * (double)m * (double)g.N * nb;
    const double bytes = (double)sizeof(T) * (2.0 * m * g.N + (double)m * nb + (double)nb * g.N);
    prof_end(st, pm, 1, bytes, flops);
    return hipSuccess;
}

template <typename T>
hipError_t launch_blocked(const T* A, int64_t n, int64_t lda, int64_t b,
                          int update, BlkWork<T> w, mc_result* out,
                          hipStream_t stream, bool factor, bool lookahead,
                          bool serialize)
{
    std::unique_lock<std::mutex> lock(g_sched_mu);
    static bool attr_set = false; // guarded by g_sched_mu
    if (!attr_set && trsm_mfma_lds_bytes<T>((int)kMaxPanel) > 64 * 1024) {
        for (const void* f : {reinterpret_cast<const void*>(&blk_trsm_mfma<T, false>),
                              reinterpret_cast<const void*>(&blk_trsm_mfma<T, true>)}) {
            const hipError_t e = hipFuncSetAttribute(
                f, hipFuncAttributeMaxDynamicSharedMemorySize,
                (int)trsm_mfma_lds_bytes<T>((int)kMaxPanel));
            if (e != hipSuccess) return note_hip_error(e);
        }
        attr_set = true;
    }
    // serialize = false: no per-device state at all (no side stream, no
    // events, no ordering against other calls) -- for callers that must not
    // have the library create runtime objects; lookahead is then off too.
    DevSched* ds = nullptr;
    if (serialize || lookahead) {
        ds = sched_get();
        if (ds == nullptr) return note_hip_error(hipErrorOutOfMemory);
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (ds) {
        const hipError_t e = hipStreamIsCapturing(stream, &cap);
        if (e != hipSuccess) return note_hip_error(e);
    }
    const bool ordered = ds != nullptr && serialize && cap == hipStreamCaptureStatusNone;
    if (ordered && ds->done_recorded) { // the device's previous blocked call
        const hipError_t e = hipStreamWaitEvent(stream, ds->done, 0);
        if (e != hipSuccess) return note_hip_error(e);
    }
    const bool split_on = g_split_on.load();
    int cus = 0; // compute units of the device (for the TRSM's spread)
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            cus < 1) {
            (void)hipGetLastError();
            cus = 256;
        }
    }
    hipLaunchKernelGGL(blk_init<T>, dim3((unsigned)n), dim3(kBlkThreads), 0,
                       stream, A, lda, n, w);
    DevSched* la = lookahead ? ds : nullptr;
    bool pending = false; // side-stream work the caller's stream must join
    bool beside = false;  // ... and it leaves XCD 0 to the next panel
    // rows of the panel starting at s0: b, except that FP64 panels wider
    // than one XCD holds at 32 columns per wavefront (8192) take at most 64
    // rows, so that the column-split panel holds 64 columns per wavefront
    // (up to 16384) instead of falling back to the row-per-block chain
    auto panel_rows = [&](int64_t s0) -> int {
        int64_t nb = std::min<int64_t>(b, n - s0);
        if (sizeof(T) == 8 && !split_fits<T>(n - s0, (int)nb, split_on) &&
            split_fits<T>(n - s0, 64, split_on))
            nb = std::min<int64_t>(nb, 64);
        return (int)nb;
    };
    int64_t last_s0 = 0, last_k = 0;
    int last_nb = 0;
    for (int64_t s0 = 0, k = 0; s0 < n; ++k) {
        const int nb = panel_rows(s0);
        const int64_t pend = s0 + nb;
        last_s0 = s0;
        last_nb = nb;
        last_k = k;
        // the panel chains need their blocks resident together on one XCD:
        // the one block 0 lands on, or XCD 0 when the trailing update
        // running beside the panel (lookahead) leaves that XCD alone
        const bool split = split_fits<T>(n - s0, nb, split_on);
        if (!split) launch_head<T>(n, s0, w, stream);
        const int ept = step_ept(n - s0);
        const bool persistent = !split && ept > 0 && nb > 1;
        const ProfMark pm = prof_begin(stream, MC_PROF_PANEL);
        if (split) { // the panel's column maps are written by the kernel
            const hipError_t e = launch_panel_split<T>(n, s0, nb, panel_view(w, k), stream,
                                                       beside);
            if (e != hipSuccess) return e;
        }
        const bool single_xcd = persistent && try_panel_x<T>(n, s0, pend, w, stream);
        if (persistent && !single_xcd) {
            switch (ept) { // wider than the single-XCD panel: across XCDs
#define MC_PANEL(E)                                                           \
    case E:                                                                   \
        hipLaunchKernelGGL((blk_panel<T, E>), dim3((unsigned)(nb - 1)),       \
                           dim3(kStepThreads), 0, stream, n, s0, pend, w);    \
        break;
                MC_PANEL(1) MC_PANEL(2) MC_PANEL(4) MC_PANEL(8) MC_PANEL(16)
#undef MC_PANEL
            }
        } else if (!persistent && !split) {
            for (int64_t s = s0; s < pend; ++s)
                launch_step<T>(n, s, s0, pend, w, stream);
        }
        { // the panel's rows read and written once; b^2 w flops
            const double width = (double)(n - s0);
            prof_end(stream, pm, (persistent || split) ? 1 : nb,
                     2.0 * sizeof(T) * nb * width, (double)nb * nb * width);
        }
        if (single_xcd) // unfactored rows; the later steps' exchanges
            hipLaunchKernelGGL(blk_fixup_x<T>, dim3((unsigned)nb),
                               dim3(kBlkThreads), 0, stream, n, s0, nb, w);
        else if (persistent) // rows published early: later exchanges
            hipLaunchKernelGGL(blk_fixup<T>, dim3((unsigned)((nb + 3) / 4)),
                               dim3(kBlkThreads), 0, stream, s0, nb, w);
        if (pend >= n) break;
        const int64_t rows = n - pend;
        const BlkWork<T> wk = panel_view(w, k);
        if (!split) // (the column-split kernel did this work itself)
            hipLaunchKernelGGL(blk_perm<T>, dim3(1), dim3(kBlkThreads), 0, stream,
                               s0, nb, wk);
        if (pending) { // the previous panel's update of the rows below
            const hipError_t e = hipStreamWaitEvent(stream, la->join, 0);
            if (e != hipSuccess) return note_hip_error(e);
            pending = false;
        }
        {
            // 16-row tiles, up to four a block, as few a block as keeps the
            // blocks within the compute units
            const int64_t tiles = (rows + 15) / 16;
            const int aw = (int)std::min<int64_t>(4, std::max<int64_t>(
                                                         1, (tiles + cus - 1) / cus));
            const dim3 grid((unsigned)((tiles + aw - 1) / aw));
            const size_t lds = trsm_mfma_lds_bytes<T>(nb);
            if (split) // inverts U11's diagonal blocks itself
                hipLaunchKernelGGL((blk_trsm_mfma<T, true>), grid, dim3(kBlkThreads), lds,
                                   stream, n, s0, nb, aw, wk);
            else
                hipLaunchKernelGGL((blk_trsm_mfma<T, false>), grid, dim3(kBlkThreads), lds,
                                   stream, n, s0, nb, aw, wk);
        }
        // lookahead, when the next panel is a column-split panel and the
        // device shows all eight XCDs: the next panel's rows first, on the
        // caller's stream, then the rest on the side stream, beside that
        // panel and leaving XCD 0 to it (tile counter zeroed by this
        // panel's TRSM or blk_perm).  Otherwise one launch for all rows:
        // beside a row-per-block panel chain the update's tiles would share
        // its XCD and slow it more than the overlap gains.
        const int next_nb = panel_rows(pend);
        beside = la && la->all_xccs && split_fits<T>(n - pend, next_nb, split_on, true) &&
                 rows > next_nb;
        const int64_t next = beside ? next_nb : rows;
        hipError_t e = trailing(wk, update, s0, nb, pend, next, n, stream, nullptr);
        if (e != hipSuccess) return e;
        hipStream_t rest = stream;
        if (beside) {
            if ((e = hipEventRecord(la->fork, stream)) != hipSuccess ||
                (e = hipStreamWaitEvent(la->side, la->fork, 0)) != hipSuccess)
                return note_hip_error(e);
            rest = la->side;
            e = trailing(wk, update, s0, nb, pend + next, rows - next, n, rest,
                         reinterpret_cast<unsigned int*>(&w.claim[2]));
            if (e != hipSuccess) return e;
        }
        if (factor) {
            hipLaunchKernelGGL(blk_store_l<T>, dim3(1024), dim3(kBlkThreads), 0,
                               rest, n, s0, nb, wk);
            if (s0 > 0)
                hipLaunchKernelGGL(blk_swaps_above<T>,
                                   dim3((unsigned)((s0 + 3) / 4)),
                                   dim3(kBlkThreads), 0, rest, s0, nb, wk);
        }
        if (rest != stream) {
            if ((e = hipEventRecord(la->join, rest)) != hipSuccess) return note_hip_error(e);
            pending = true;
        }
        s0 = pend;
    }
    if (pending) {
        const hipError_t e = hipStreamWaitEvent(stream, la->join, 0);
        if (e != hipSuccess) return note_hip_error(e);
    }
    // the last panel (no rows below): its exchanges still reach the rows
    // above it in factor mode
    if (factor && n > 0) {
        const int64_t s0 = last_s0;
        const int nb = last_nb;
        if (s0 > 0) {
            const BlkWork<T> wk = panel_view(w, last_k);
            hipLaunchKernelGGL(blk_perm<T>, dim3(1), dim3(kBlkThreads), 0, stream,
                               s0, nb, wk);
            hipLaunchKernelGGL(blk_swaps_above<T>, dim3((unsigned)((s0 + 3) / 4)),
                               dim3(kBlkThreads), 0, stream, s0, nb, wk);
        }
    }
    hipLaunchKernelGGL(blk_finalize, dim3(1), dim3(kBlkThreads), 0, stream, n,
                       w.piv_pos, w.piv_val, w.state, out);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ordered) {
        const hipError_t e = hipEventRecord(ds->done, stream);
        if (e != hipSuccess) return note_hip_error(e);
        ds->done_recorded = true;
    }
    return hipSuccess;
}

template hipError_t launch_blocked<double>(const double*, int64_t, int64_t,
                                           int64_t, int, BlkWork<double>,
                                           mc_result*, hipStream_t, bool, bool,
                                           bool);
template hipError_t launch_blocked<float>(const float*, int64_t, int64_t,
                                          int64_t, int, BlkWork<float>,
                                          mc_result*, hipStream_t, bool, bool,
                                          bool);

} // namespace mc
