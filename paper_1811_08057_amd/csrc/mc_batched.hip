// mc_batched.hip -- many matrices of uneven sizes in one persistent launch.
//
// Use case: the log-determinants of many covariance matrices, e.g. the
// components of a mixture model (Abstract).  Each workgroup repeatedly takes
// the next matrix from an atomic queue ordered largest first and condenses
// it alone: the blocked algorithm of mc_blocked.hip (panel steps with the
// largest-|a| pivot and row factoring, gathered triangular solve, trailing
// update on the matrix cores) expressed at workgroup level, with the
// matrix in its own region of the workspace.  A setup kernel resets the
// queue and orders the batch; the two kernels are the whole call, so a
// caller can capture it in a hipGraph.
//
// Panel width b and the trailing-update tile come from a small table keyed
// by size bucket (filled by mc_autotune_batched, or defaults).
#include <algorithm>
#include <atomic>

#include "mc_batched.h"
#include "mc_device.h"
#include "mc_mfma.h"

namespace mc {

constexpr int kBT = 256; // threads per workgroup (4 wavefronts)

__host__ __device__ inline int bucket_of(int64_t n)
{
    int k = 0;
    while (k < kTuneBuckets - 1 && n > tune_bucket_max(k)) ++k;
    return k;
}

__host__ __device__ inline int64_t bat_ldw(int64_t n, int elem)
{
    const int64_t per = 128 / elem;
    return (n + per - 1) / per * per;
}

__host__ __device__ inline size_t bat_align(size_t x) { return (x + 255) / 256 * 256; }

// Bytes of one matrix's region for size n and panel width b (the factor
// call works on the caller's matrix in place and keeps no copy W).
__host__ __device__ inline size_t bat_region_bytes(int64_t n, int64_t b, int elem,
                                                   bool with_w = true)
{
    const size_t nblk = (size_t)((b + 15) / 16);
    size_t t = 0;
    if (with_w) t += bat_align((size_t)elem * (size_t)n * (size_t)bat_ldw(n, elem)); // W
    t += bat_align((size_t)elem * (size_t)n * (size_t)b);               // L
    t += 3 * bat_align(sizeof(int) * (size_t)n);   // piv_pos, perm, colsrc
    t += bat_align(sizeof(double) * (size_t)n);    // piv_val
    t += bat_align(sizeof(int) * (size_t)b);       // srcp
    t += bat_align((size_t)elem * nblk * 256);     // dinv
    return t;
}

template <typename T>
struct Region {
    T* W;
    int64_t ldw;
    T* L;
    int* piv_pos;
    int* perm;
    int* colsrc;
    double* piv_val;
    int* srcp;
    T* dinv;
};

template <typename T>
__device__ inline Region<T> carve_region(unsigned char* base, int64_t n,
                                         int64_t b, bool with_w = true)
{
    Region<T> r;
    const int elem = (int)sizeof(T);
    r.ldw = bat_ldw(n, elem);
    unsigned char* p = base;
    auto take = [&](size_t bytes) {
        unsigned char* q = p;
        p += bat_align(bytes);
        return q;
    };
    r.W = with_w ? reinterpret_cast<T*>(take((size_t)elem * n * r.ldw)) : nullptr;
    r.L = reinterpret_cast<T*>(take((size_t)elem * n * b));
    r.piv_pos = reinterpret_cast<int*>(take(sizeof(int) * n));
    r.perm = reinterpret_cast<int*>(take(sizeof(int) * n));
    r.colsrc = reinterpret_cast<int*>(take(sizeof(int) * n));
    r.piv_val = reinterpret_cast<double*>(take(sizeof(double) * n));
    r.srcp = reinterpret_cast<int*>(take(sizeof(int) * b));
    r.dinv = reinterpret_cast<T*>(take((size_t)elem * ((b + 15) / 16) * 256));
    return r;
}

// ------------------------------------------------------------------ setup

// One block: reset the queue and rank the matrices by size, largest first
// (ties by index), so big matrices start early and small ones fill in.
// (Batches larger than kSortMax keep their given order.)
constexpr int64_t kSortMax = 16384;

__global__ void __launch_bounds__(kBT)
batched_setup(const int64_t* __restrict__ n_array, int64_t batch, int* counter,
              int* order)
{
    if (threadIdx.x == 0) *counter = 0;
    if (batch > kSortMax) {
        for (int64_t i = threadIdx.x; i < batch; i += kBT) order[i] = (int)i;
        return;
    }
    for (int64_t i = threadIdx.x; i < batch; i += kBT) {
        const int64_t ni = n_array[i];
        int64_t rank = 0;
        for (int64_t j = 0; j < batch; ++j) {
            const int64_t nj = n_array[j];
            rank += (nj > ni || (nj == ni && j < i)) ? 1 : 0;
        }
        order[rank] = (int)i;
    }
}

// --------------------------------------------------------- workgroup stages

struct WgShared {
    PivotKey keys[kBT / kWave];
    int flag;
    int status;
    int piv_slot;
    int qidx;
    double piv;
    double vs;
    double csum[kBT];
    double ccomp[kBT];
    int cpar[kBT];
};

// Argmax of row s over positions [s, n), record the pivot, factor the row
// (position s <- p, position l <- old(s)/p, others /p).  Returns the status.
template <typename T>
__device__ int wg_pivot_row(Region<T>& r, int64_t n, int64_t s, WgShared& sh)
{
    const int tid = threadIdx.x;
    T* row = r.W + s * r.ldw;
    PivotKey k = no_candidate();
    bool bad = false;
    for (int64_t j = s + tid; j < n; j += kBT) {
        const T v = row[j];
        if (j == s) sh.vs = (double)v;
        if (!offer(k, (double)v, r.perm[j], (int)j)) bad = true;
    }
    k = block_argmax<kBT>(k, bad, sh.keys, &sh.flag);
    int st = kStatusOk;
    if (bad)
        st = kStatusNonfinite;
    else if (k.slot < 0 || k.value == 0.0)
        st = kStatusSingular;
    if (tid == 0) {
        r.piv_pos[s] = k.slot;
        r.piv_val[s] = k.value;
        if (st == kStatusOk) {
            const int a = r.perm[s];
            r.perm[s] = r.perm[k.slot];
            r.perm[k.slot] = a;
        }
    }
    if (st == kStatusOk) {
        const T p = (T)k.value;
        const T vs = (T)sh.vs;
        const int64_t l = k.slot;
        for (int64_t j = s + tid; j < n; j += kBT) {
            const T v = row[j];
            row[j] = (j == s) ? p : ((j == l) ? vs : v) / p;
        }
    }
    __syncthreads();
    return st;
}

// Rows through buffer descriptors: a position past the row (or any
// position of a zero-length row) reads 0 and a store there is dropped, so a
// thread's loads go out together, with no branch between them.
constexpr uint32_t kPastRow = 0x7ffffff0u;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T* row, int64_t len)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(row), 0, (int)(sizeof(T) * len),
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ T row_load(__amdgpu_buffer_rsrc_t r, int64_t j, int64_t len)
{
    return operand_load<T>(r, j < len ? (uint32_t)(sizeof(T) * j) : kPastRow);
}

__device__ __forceinline__ void row_store(double v, __amdgpu_buffer_rsrc_t r, int64_t j,
                                          int64_t len)
{
    typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u32, v), r,
                                          j < len ? (uint32_t)(8 * j) : kPastRow, 0, 0);
}

__device__ __forceinline__ void row_store(float v, __amdgpu_buffer_rsrc_t r, int64_t j,
                                          int64_t len)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r,
                                          j < len ? (uint32_t)(4 * j) : kPastRow, 0, 0);
}

// The later panel rows' update of step s (rows s+1.., R of them): a
// thread takes columns s+1+tid+q kBT (q < QC) of every row, rows in groups
// of RG whose loads go out together, the next group's loads in flight while
// this group's results are stored.  QC x RG = 16 loads a group: fewer
// columns a thread (shorter rows) take more rows a group.  sc, sx: each
// row's entry at l and its old entry at s (already staged).
template <typename T, int QC, int RG>
__device__ void panel_rows_update(T* W, int64_t ldw, int64_t n, int64_t s, int64_t l, int R,
                                  const T* sc, const T* sx)
{
    const int tid = threadIdx.x;
    const __amdgpu_buffer_rsrc_t rrs = row_rsrc(W + s * ldw, n);
    for (int64_t jb = s + 1 + tid; jb < n; jb += QC * kBT) {
        T rv[QC];
#pragma unroll
        for (int q = 0; q < QC; ++q) rv[q] = row_load<T>(rrs, jb + q * kBT, n);
        auto rrow = [&](int i) { // row s+1+i, or nothing past the panel
            return row_rsrc(W + (s + 1 + (i < R ? i : 0)) * ldw, i < R ? n : 0);
        };
        auto load_group = [&](int i0, T (&xv)[RG][QC]) {
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const __amdgpu_buffer_rsrc_t rr = rrow(i0 + g);
#pragma unroll
                for (int q = 0; q < QC; ++q) xv[g][q] = row_load<T>(rr, jb + q * kBT, n);
            }
        };
        auto store_group = [&](int i0, const T (&xv)[RG][QC]) {
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int i = i0 + g;
                const __amdgpu_buffer_rsrc_t rr = rrow(i);
                const T c = sc[i < R ? i : 0], xs = sx[i < R ? i : 0];
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int64_t j = jb + q * kBT;
                    row_store(fma(-c, rv[q], (j == l) ? xs : xv[g][q]), rr, j, n);
                }
            }
        };
        T xa[RG][QC], xb[RG][QC];
        load_group(0, xa);
        for (int i0 = 0; i0 < R; i0 += 2 * RG) {
            if (i0 + RG < R) load_group(i0 + RG, xb);
            store_group(i0, xa);
            if (i0 + 2 * RG < R) load_group(i0 + 2 * RG, xa);
            if (i0 + RG < R) store_group(i0 + RG, xb);
        }
    }
}

// Step s inside the panel [s0, pend): exchange positions s, l in the
// earlier rows (the panel's own, or every row above when the factors are
// kept: rows above hold U entries there); update the later panel rows:
// row i's position s takes c_i (its entry at l: the pivot column moves to
// s), position l the old entry at s, and every position j > s loses c_i
// times the factored pivot row's entry.  Short rows (at most kBT
// positions right of s): one wavefront a row, the lanes along it (two
// round trips a row at most); longer rows: the grouped form above, after
// each row's entries at l and s are staged in `lds` (2 kMaxPanel elements).
template <typename T>
__device__ void wg_panel_update(Region<T>& r, int64_t n, int64_t s,
                                int64_t s0, int64_t pend, int64_t l,
                                bool factor, T* lds)
{
    const int tid = threadIdx.x;
    T* W = r.W;
    const int64_t ldw = r.ldw;
    if (l != s)
        for (int64_t u = (factor ? 0 : s0) + tid; u < s; u += kBT) {
            T* ru = W + u * ldw;
            const T a = ru[s];
            ru[s] = ru[l];
            ru[l] = a;
        }
    const int64_t cols = n - s - 1;
    if (cols <= kBT) {
        const int lane = tid & 63, wid = tid >> 6;
        const T* rs = W + s * ldw;
        for (int64_t i = s + 1 + wid; i < pend; i += kBT / kWave) {
            T* ri = W + i * ldw;
            const T c = ri[l]; // every lane reads it before any lane writes
            for (int64_t j = s + 1 + lane; j < n; j += kWave) {
                T x;
                if (j == l) {
                    x = ri[s];
                    ri[s] = c;
                } else {
                    x = ri[j];
                }
                ri[j] = fma(-c, rs[j], x);
            }
        }
        __syncthreads();
        return;
    }
    const int R = (int)(pend - s - 1); // later panel rows
    T* sc = lds;
    T* sx = lds + kMaxPanel;
    if (tid < R) {
        T* ri = W + (s + 1 + tid) * ldw;
        const T c = ri[l];
        sx[tid] = ri[s];
        sc[tid] = c;
        ri[s] = c;
    }
    __syncthreads();
    if (cols <= 2 * kBT)
        panel_rows_update<T, 2, 8>(W, ldw, n, s, l, R, sc, sx);
    else
        panel_rows_update<T, 4, 4>(W, ldw, n, s, l, R, sc, sx);
    __syncthreads();
}

// Sources of the moved columns for the rows below the panel, and the
// inverses of U11's 16 x 16 diagonal blocks (as blk_perm).
template <typename T>
__device__ void wg_perm(Region<T>& r, int64_t n, int64_t s0, int nb)
{
    const int tid = threadIdx.x;
    const int64_t pend = s0 + nb;
    for (int64_t j = pend + tid; j < n; j += kBT) r.colsrc[j] = (int)j;
    __syncthreads();
    auto trace = [&](int64_t d) -> int {
        int64_t pos = d;
        for (int u = nb - 1; u >= 0; --u) {
            const int64_t a = s0 + u, b = r.piv_pos[s0 + u];
            if (pos == a)
                pos = b;
            else if (pos == b)
                pos = a;
        }
        return (int)pos;
    };
    for (int t = tid; t < nb; t += kBT) {
        r.srcp[t] = trace(s0 + t);
        const int64_t d = r.piv_pos[s0 + t];
        if (d >= pend) r.colsrc[d] = trace(d);
    }
    const int nblk = (nb + 15) / 16;
    const T* U = r.W + s0 * r.ldw + s0;
    for (int e = tid; e < nblk * 16; e += kBT) {
        const int J = e >> 4, c = e & 15;
        T x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = (q == c) ? T(1) : T(0);
#pragma unroll
        for (int q = 14; q >= 0; --q) {
            if (q >= c) continue;
            T sum = 0;
#pragma unroll
            for (int v = q + 1; v < 16; ++v) {
                if (v > c) break;
                const int pv = 16 * J + v;
                const T u = (pv < nb) ? U[(int64_t)(16 * J + q) * r.ldw + pv] : T(0);
                sum = fma(u, x[v], sum);
            }
            x[q] = -sum;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) r.dinv[(J * 16 + q) * 16 + c] = x[q];
    }
    __syncthreads();
}

// L21 = A21 * U11^{-1} for the rows below the panel on the matrix cores,
// as its transpose X^T = U11^{-T} A21^T in 16-row blocks J of X^T:
//     R_J = A21^T[J, :] - sum_{K<J} U11[K, J]^T X^T[K, :]
//     X^T[J, :] = inv(U11[J, J])^T R_J
// (A21[i][t] = W[i][srcp[t]], the exchanges folded into the load).  Each
// wavefront takes 16 rows at a time; a finished block, in the accumulator
// layout, is already the second operand of the later blocks' products (the
// rows of X^T a lane holds are the k values it supplies), so X never leaves
// the registers and the row loop has no barrier.  U11's strictly upper
// 16 x 16 blocks, the inverted diagonal blocks (wg_perm) and the columns'
// sources are staged in LDS first; A21's entries come through a buffer
// descriptor (rows past n read zero), all of a row group's in flight
// together.  MB: the most 16-column blocks the panel may have.
template <typename T, int MB>
__device__ void wg_trsm_blocks(Region<T>& r, int64_t n, int64_t s0, int nb, T* lds)
{
    using P = typename MfmaFor<T>::P;
    constexpr int kTri = MB * (MB - 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nblk = (nb + 15) / 16;
    const int ntri = nblk * (nblk - 1) / 2;
    T* Ub = lds;                 // block (K, J), K < J, at tri(K, J) = J (J - 1) / 2 + K
    T* Dv = lds + ntri * 256;    // inv(U11[J, J]), row-major per block
    int* src = reinterpret_cast<int*>(Dv + nblk * 256); // 16 nblk sources
    const int64_t pend = s0 + nb, m = n - pend;
    const int64_t ldw = r.ldw;
    const int cin = lane & 15;
    {
        const int er = tid >> 4, ec = tid & 15;
        const __amdgpu_buffer_rsrc_t ru = operand_rsrc(
            r.W + s0 * ldw + s0, (int64_t)sizeof(T) * ((int64_t)(nb - 1) * ldw + nb));
        // item u < kTri: upper block tri(K, J) = u; else diagonal block
        // u - kTri; in chunks of CH items (loads of a chunk in flight
        // together, the chunks one after another: the registers hold one)
        constexpr int NI = kTri + MB, CH = NI <= 12 ? NI : 9;
#pragma unroll
        for (int c0 = 0; c0 < NI; c0 += CH) {
            T v[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int it = c0 + u;
                if (it >= NI) break;
                if (it < kTri) {
                    int J = 1;
                    while (J * (J + 1) / 2 <= it) ++J; // tri(K, J) = it
                    const int K = it - J * (J - 1) / 2, t = 16 * J + ec;
                    // row 16 K + er < nb whenever K < J < nblk
                    v[u] = operand_load<T>(
                        ru, (J < nblk && t < nb)
                                ? (uint32_t)(sizeof(T) * ((16 * K + er) * ldw + t))
                                : kOutOfRange);
                } else {
                    const int J = it - kTri;
                    v[u] = J < nblk ? r.dinv[J * 256 + tid] : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int it = c0 + u;
                if (it >= NI) break;
                if (it < kTri) {
                    int J = 1;
                    while (J * (J + 1) / 2 <= it) ++J;
                    if (J < nblk) Ub[it * 256 + tid] = v[u];
                } else if (it - kTri < nblk) {
                    Dv[(it - kTri) * 256 + tid] = v[u];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (tid < 16 * nblk) src[tid] = tid < nb ? r.srcp[tid] : 0;
    }
    __syncthreads();
    for (int64_t g0 = 0; g0 < m; g0 += 64) {
        // lane (cin, q) of block J: row g0 + li (from pend), column
        // 16 J + P::drow(lane, q); one descriptor per group of 64 rows keeps
        // the offsets small for any matrix
        const int li = wid * 16 + cin;
        const int64_t i = g0 + li;
        const bool rin = i < m;
        const __amdgpu_buffer_rsrc_t ra = operand_rsrc(
            r.W + (pend + g0) * ldw, (int64_t)sizeof(T) * (m - g0 < 64 ? m - g0 : 64) * ldw);
        // up to 4 blocks, every entry first; beyond (panels wider than 64
        // columns, only on request) each block's entries at that block, so
        // that the registers hold one block of them
        constexpr bool kAll = MB <= 4;
        auto gather = [&](int J, T* gj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 16 * J + P::drow(lane, q);
                gj[q] = operand_load<T>(
                    ra, (rin && J < nblk && t < nb)
                            ? (uint32_t)(sizeof(T) * ((int64_t)li * ldw + src[t]))
                            : kOutOfRange);
            }
        };
        T g[kAll ? MB : 1][4];
        if (kAll) {
#pragma unroll
            for (int J = 0; J < MB; ++J) gather(J, g[kAll ? J : 0]);
        }
        typename P::Acc xt[MB];
#pragma unroll
        for (int J = 0; J < MB; ++J) {
            if (J >= nblk) break;
            if (!kAll) gather(J, g[0]);
            typename P::Acc acc;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = g[kAll ? J : 0][q];
#pragma unroll
            for (int K = 0; K < MB; ++K) {
                if (K >= J) break;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T a = -Ub[(J * (J - 1) / 2 + K) * 256 + P::drow(lane, q) * 16 + cin];
                    acc = P::mma(a, xt[K][q], acc);
                }
            }
            typename P::Acc x = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                x = P::mma(Dv[(J * 16 + P::drow(lane, q)) * 16 + cin], acc[q], x);
            xt[J] = x;
        }
        if (rin) {
            T* lrow = r.L + i * nb;
#pragma unroll
            for (int J = 0; J < MB; ++J) {
                if (J >= nblk) break;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t = 16 * J + P::drow(lane, q);
                    if (t < nb) lrow[t] = xt[J][q];
                }
            }
        }
    }
    __syncthreads(); // the LDS is the trailing update's next
}

template <typename T>
__device__ void wg_trsm(Region<T>& r, int64_t n, int64_t s0, int nb, T* lds)
{
    if (nb <= 64)
        wg_trsm_blocks<T, 4>(r, n, s0, nb, lds);
    else
        wg_trsm_blocks<T, (int)(kMaxPanel / 16)>(r, n, s0, nb, lds);
}

// Trailing update C[pend:, pend:] <- C[., colsrc] - L U12 with tiles of
// (32 TM) x (32 TN): 4 wavefronts in 2 x 2, TM x TN MFMA tiles each.  The
// K loop is double-buffered: chunk c+1 is read into registers (buffer
// loads, out-of-range entries reading 0, all in flight at once) while chunk
// c feeds the matrix cores, then parked in the other LDS buffer; the tile's
// old C is read behind chunk 1's operands, so the epilogue waits on no load.
template <typename T, int TM, int TN>
__device__ void wg_gemm_scalar(Region<T>& r, int64_t n, int64_t s0, int nb,
                               T* lds)
{
    using P = typename MfmaFor<T>::P;
    constexpr int BM = 32 * TM, BN = 32 * TN;
    constexpr int KC = 16;
    constexpr int LDA = BM + 16, LDB = BN + 16;
    constexpr int PA = (BM * KC + kBT - 1) / kBT; // elements of A per thread per chunk
    constexpr int PB = (BN * KC + kBT - 1) / kBT;
    T* As = lds;                 // [2][KC][LDA]
    T* Bs = lds + 2 * KC * LDA;  // [2][KC][LDB]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int cin = lane & 15, kl = lane >> 4;
    const int64_t pend = s0 + nb, M = n - pend;
    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (M + BN - 1) / BN;
    const int nch = (nb + KC - 1) / KC;
    const __amdgpu_buffer_rsrc_t rcs = operand_rsrc(r.colsrc + pend, sizeof(int) * M);
    for (int64_t t = 0; t < tiles_m * tiles_n; ++t) {
        const int64_t rb = (t / tiles_n) * BM, cb = (t % tiles_n) * BN;
        // the tile's rows of L (M x nb, row stride nb) and of C, and U12's
        // nb rows from the tile's first column (offsets stay below 2^31
        // bytes for any matrix that fits in memory)
        const int64_t rows = (M - rb) < BM ? (M - rb) : BM;
        const __amdgpu_buffer_rsrc_t rl = operand_rsrc(r.L + rb * nb, sizeof(T) * rows * nb);
        const __amdgpu_buffer_rsrc_t ru = operand_rsrc(
            r.W + s0 * r.ldw + pend + cb, sizeof(T) * ((int64_t)(nb - 1) * r.ldw + (M - cb)));
        const __amdgpu_buffer_rsrc_t rcm =
            operand_rsrc(r.W + (pend + rb) * r.ldw, sizeof(T) * rows * r.ldw);
        T pa[PA], pb[PB];
        auto gload = [&](int k0) {
#pragma unroll
            for (int p = 0; p < PA; ++p) {
                const int e = tid + p * kBT;
                const int rr = e / KC, kk = e - rr * KC;
                const bool oka = e < BM * KC && k0 + kk < nb; // rows past M: past the range
                pa[p] = operand_load<T>(
                    rl, oka ? (uint32_t)(sizeof(T) * (rr * nb + k0 + kk)) : kOutOfRange);
            }
#pragma unroll
            for (int p = 0; p < PB; ++p) {
                const int e = tid + p * kBT;
                const int kb = e / BN, cc = e - kb * BN;
                const bool okb = e < BN * KC && cb + cc < M && k0 + kb < nb;
                pb[p] = operand_load<T>(
                    ru, okb ? (uint32_t)(sizeof(T) * ((int64_t)(k0 + kb) * r.ldw + cc))
                            : kOutOfRange);
            }
        };
        auto sstore = [&](int buf) {
#pragma unroll
            for (int p = 0; p < PA; ++p) {
                const int e = tid + p * kBT;
                const int rr = e / KC, kk = e - rr * KC;
                if (e < BM * KC) As[(buf * KC + kk) * LDA + rr] = -pa[p];
            }
#pragma unroll
            for (int p = 0; p < PB; ++p) {
                const int e = tid + p * kBT;
                const int kb = e / BN, cc = e - kb * BN;
                if (e < BN * KC) Bs[(buf * KC + kb) * LDB + cc] = pb[p];
            }
        };
        int csrc[TN];
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            const int64_t col = cb + wn * 16 * TN + tj * 16 + cin;
            csrc[tj] = (int)__builtin_amdgcn_raw_buffer_load_b32(
                rcs, col < M ? (uint32_t)(sizeof(int) * col) : kOutOfRange, 0, 0);
        }
        gload(0);
        typename P::Acc acc[TM][TN];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[a][b][q] = T(0);
        sstore(0);
        __syncthreads();
        T cpre[TM][TN][4];
        for (int c = 0; c < nch; ++c) {
            const int buf = c & 1;
            if (c + 1 < nch) gload((c + 1) * KC);
            if (c == 0) {
#pragma unroll
                for (int tj = 0; tj < TN; ++tj) {
                    const bool okc = cb + wn * 16 * TN + tj * 16 + cin < M;
#pragma unroll
                    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int rr = wm * 16 * TM + ti * 16 + P::drow(lane, q);
                            cpre[ti][tj][q] = operand_load<T>(
                                rcm, okc ? (uint32_t)(sizeof(T) * (rr * r.ldw + csrc[tj]))
                                         : kOutOfRange);
                        }
                }
            }
#pragma unroll
            for (int kq = 0; kq < KC; kq += 4) {
                T a[TM], b[TN];
#pragma unroll
                for (int q = 0; q < TM; ++q)
                    a[q] = As[(buf * KC + kq + kl) * LDA + wm * 16 * TM + q * 16 + cin];
#pragma unroll
                for (int q = 0; q < TN; ++q)
                    b[q] = Bs[(buf * KC + kq + kl) * LDB + wn * 16 * TN + q * 16 + cin];
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int tj = 0; tj < TN; ++tj)
                        acc[ti][tj] = P::mma(a[ti], b[tj], acc[ti][tj]);
            }
            if (c + 1 < nch) sstore(buf ^ 1);
            __syncthreads();
        }
        // C[dst] = C[src] + acc (a moved column's source lies in the
        // panel's column range, which no tile writes)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            const int64_t col = cb + wn * 16 * TN + tj * 16 + cin;
            if (col >= M) continue;
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t row = rb + wm * 16 * TM + ti * 16 + P::drow(lane, q);
                    if (row < M)
                        r.W[(pend + row) * r.ldw + pend + col] = cpre[ti][tj][q] + acc[ti][tj][q];
                }
        }
    }
    __syncthreads();
}

// With a 64-wide tile chosen, trailing blocks of at least this many rows
// take 128 x 64 tiles (each wavefront 64 x 32: eight accumulators, so more
// independent products per operand read at one wavefront per SIMD).
constexpr int64_t kBigTileRows = 512;

// Split-BF16 x 3 form of the trailing update (FP32 storage).
template <int WT>
__device__ void wg_gemm_bf16x3(Region<float>& r, int64_t n, int64_t s0, int nb,
                               float* lds_f)
{
    constexpr int BT = 32 * WT;
    constexpr int KC = 32;
    constexpr int LD = KC + 8;
    __bf16* Ah = reinterpret_cast<__bf16*>(lds_f);
    __bf16* Al = Ah + BT * LD;
    __bf16* Bh = Al + BT * LD;
    __bf16* Bl = Bh + BT * LD;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int cin = lane & 15, kg = lane >> 4;
    const int64_t pend = s0 + nb, M = n - pend;
    const int64_t tiles = (M + BT - 1) / BT;
    const float* U = r.W + s0 * r.ldw;
    for (int64_t t = 0; t < tiles * tiles; ++t) {
        const int64_t rb = (t / tiles) * BT, cb = (t % tiles) * BT;
        f4 acc[WT][WT];
#pragma unroll
        for (int a = 0; a < WT; ++a)
#pragma unroll
            for (int b = 0; b < WT; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < nb; k0 += KC) {
            for (int e = tid; e < BT * KC; e += kBT) {
                const int rr = e / KC, kk = e - rr * KC;
                const int64_t row = rb + rr;
                const float va = (row < M && k0 + kk < nb)
                                     ? -r.L[row * nb + k0 + kk]
                                     : 0.0f;
                const __bf16 ha = (__bf16)va;
                Ah[rr * LD + kk] = ha;
                Al[rr * LD + kk] = (__bf16)(va - (float)ha);
                const int kb = e / BT, cc = e - kb * BT;
                const int64_t col = cb + cc;
                const float vb = (col < M && k0 + kb < nb)
                                     ? U[(int64_t)(k0 + kb) * r.ldw + pend + col]
                                     : 0.0f;
                const __bf16 hb = (__bf16)vb;
                Bh[cc * LD + kb] = hb;
                Bl[cc * LD + kb] = (__bf16)(vb - (float)hb);
            }
            __syncthreads();
            bf8 ah[WT], al[WT], bh[WT], bl[WT];
#pragma unroll
            for (int q = 0; q < WT; ++q) {
                const int ar = wm * 16 * WT + q * 16 + cin;
                const int bc = wn * 16 * WT + q * 16 + cin;
                ah[q] = *reinterpret_cast<const bf8*>(&Ah[ar * LD + 8 * kg]);
                al[q] = *reinterpret_cast<const bf8*>(&Al[ar * LD + 8 * kg]);
                bh[q] = *reinterpret_cast<const bf8*>(&Bh[bc * LD + 8 * kg]);
                bl[q] = *reinterpret_cast<const bf8*>(&Bl[bc * LD + 8 * kg]);
            }
#pragma unroll
            for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                for (int tj = 0; tj < WT; ++tj) {
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        al[ti], bh[tj], acc[ti][tj], 0, 0, 0);
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        ah[ti], bl[tj], acc[ti][tj], 0, 0, 0);
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        ah[ti], bh[tj], acc[ti][tj], 0, 0, 0);
                }
            __syncthreads();
        }
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) {
            const int64_t col = cb + wn * 16 * WT + tj * 16 + cin;
            if (col >= M) continue;
            const int64_t src = r.colsrc[pend + col];
#pragma unroll
            for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t row = rb + wm * 16 * WT + ti * 16 + 4 * kg + q;
                    if (row < M) {
                        float* crow = r.W + (pend + row) * r.ldw;
                        crow[pend + col] = crow[src] + acc[ti][tj][q];
                    }
                }
        }
    }
    __syncthreads();
}

template <typename T>
__device__ void wg_trailing(Region<T>& r, int64_t n, int64_t s0, int nb,
                            int tile, int update, T* lds);

template <>
__device__ void wg_trailing<double>(Region<double>& r, int64_t n, int64_t s0,
                                    int nb, int tile, int update, double* lds)
{
    (void)update;
    if (tile >= 64 && n - s0 - nb >= kBigTileRows)
        wg_gemm_scalar<double, 4, 2>(r, n, s0, nb, lds);
    else if (tile >= 64)
        wg_gemm_scalar<double, 2, 2>(r, n, s0, nb, lds);
    else
        wg_gemm_scalar<double, 1, 1>(r, n, s0, nb, lds);
}

template <>
__device__ void wg_trailing<float>(Region<float>& r, int64_t n, int64_t s0,
                                   int nb, int tile, int update, float* lds)
{
    if (update == MC_UPDATE_BF16X3) {
        if (tile >= 64)
            wg_gemm_bf16x3<2>(r, n, s0, nb, lds);
        else
            wg_gemm_bf16x3<1>(r, n, s0, nb, lds);
    } else {
        if (tile >= 64 && n - s0 - nb >= kBigTileRows)
            wg_gemm_scalar<float, 4, 2>(r, n, s0, nb, lds);
        else if (tile >= 64)
            wg_gemm_scalar<float, 2, 2>(r, n, s0, nb, lds);
        else
            wg_gemm_scalar<float, 1, 1>(r, n, s0, nb, lds);
    }
}

// Whole condensation of one matrix by one workgroup.  With `perm_out`
// (the factor call) the matrix A is condensed in place and keeps L\U as
// mc_logdet_factor leaves it: A_in[:, perm] = L U, the multipliers of each
// panel's rows below it stored at the panel's positions after its trailing
// update, every exchange applied to the rows above.
template <typename T>
__device__ void wg_factor(const T* __restrict__ A, int64_t n, int64_t lda,
                          int64_t b, int tile, int update,
                          unsigned char* region, mc_result* out, WgShared& sh,
                          T* lds, int32_t* perm_out)
{
    const bool factor = perm_out != nullptr;
    const int tid = threadIdx.x;
    if (n == 0) {
        if (tid == 0) {
            out->logabsdet = 0.0;
            out->sign = 1.0;
            out->info = 0;
        }
        return;
    }
    Region<T> r = carve_region<T>(region, n, b, !factor);
    if (factor) {
        r.W = const_cast<T*>(A);
        r.ldw = lda;
        r.perm = perm_out;
    } else {
        for (int64_t i = tid >> 6; i < n; i += kBT / kWave)
            for (int64_t j = tid & 63; j < n; j += kWave)
                r.W[i * r.ldw + j] = A[i * lda + j];
    }
    for (int64_t j = tid; j < n; j += kBT) r.perm[j] = (int)j;
    __syncthreads();

    int st = kStatusOk;
    int64_t bad_step = 0;
    for (int64_t s0 = 0; s0 < n && st == kStatusOk; s0 += b) {
        const int nb = (int)((b < n - s0) ? b : (n - s0));
        const int64_t pend = s0 + nb;
        st = wg_pivot_row<T>(r, n, s0, sh);
        if (st != kStatusOk) {
            bad_step = s0;
            break;
        }
        for (int64_t s = s0; s < pend; ++s) {
            const int64_t l = r.piv_pos[s];
            wg_panel_update<T>(r, n, s, s0, pend, l, factor, lds);
            if (s + 1 < pend) {
                st = wg_pivot_row<T>(r, n, s + 1, sh);
                if (st != kStatusOk) {
                    bad_step = s + 1;
                    break;
                }
            }
        }
        if (st != kStatusOk || pend >= n) break;
        wg_perm<T>(r, n, s0, nb);
        wg_trsm<T>(r, n, s0, nb, lds);
        wg_trailing<T>(r, n, s0, nb, tile, update, lds);
        if (factor) { // L21 to the panel's positions (the update read them)
            for (int64_t e = tid; e < (n - pend) * nb; e += kBT) {
                const int64_t row = pend + e / nb;
                const int t = (int)(e % nb);
                r.W[row * r.ldw + s0 + t] = r.L[(row - pend) * nb + t];
            }
            __syncthreads();
        }
    }

    // compensated sum of log|p| and sign parity (as blk_finalize)
    if (st != kStatusOk) {
        if (tid == 0) {
            const bool sing = st == kStatusSingular;
            out->logabsdet = sing ? -INFINITY : NAN;
            out->sign = 0.0;
            out->info = sing ? bad_step + 1 : (int64_t)MC_INFO_NONFINITE;
        }
        __syncthreads();
        return;
    }
    Compensated acc{0.0, 0.0};
    int par = 0;
    for (int64_t s = tid; s < n; s += kBT) {
        const double p = r.piv_val[s];
        comp_add(acc, log(fabs(p)));
        par ^= (p < 0.0) ? 1 : 0;
        par ^= (r.piv_pos[s] != (int)s) ? 1 : 0;
    }
    sh.csum[tid] = acc.sum;
    sh.ccomp[tid] = acc.comp;
    sh.cpar[tid] = par;
    __syncthreads();
    if (tid == 0) {
        Compensated tot{0.0, 0.0};
        int pp = 0;
        for (int t = 0; t < kBT; ++t) {
            comp_merge(tot, Compensated{sh.csum[t], sh.ccomp[t]});
            pp ^= sh.cpar[t];
        }
        const double la = tot.sum + tot.comp;
        if (!isfinite(la)) {
            out->logabsdet = NAN;
            out->sign = 0.0;
            out->info = MC_INFO_NONFINITE;
        } else {
            out->logabsdet = la;
            out->sign = pp ? -1.0 : 1.0;
            out->info = 0;
        }
    }
    __syncthreads();
}

// The persistent kernel: grid = resident workgroups; each loops over the
// queue until it is empty.  Every workgroup reaches the exit.
template <typename T>
__global__ void __launch_bounds__(kBT)
batched_persistent(BatchArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ WgShared sh;
    T* lds = reinterpret_cast<T*>(smem_raw);
    if (a.skip_xcc0 && xcc_id() == 0) return; // before taking any matrix
    for (;;) {
        if (threadIdx.x == 0) sh.qidx = atomicAdd(a.counter, 1);
        __syncthreads();
        const int q = sh.qidx;
        __syncthreads();
        if (q >= a.batch) break;
        const int k = a.order[q];
        const int64_t n = a.n_array[k];
        if (n < 0 || n > a.n_max || a.lda_array[k] < (n > 1 ? n : 1) ||
            (n > 0 && a.A_array[k] == nullptr)) {
            if (threadIdx.x == 0) {
                a.out[k].logabsdet = NAN;
                a.out[k].sign = 0.0;
                a.out[k].info = MC_INFO_BADARG;
            }
            continue;
        }
        const int bk = bucket_of(n);
        const int64_t b = a.table.b[bk];
        const int tile = a.table.tile[bk];
        unsigned char* region = a.regions + (size_t)k * a.region_stride;
        int32_t* perm = a.perm_array ? a.perm_array[k] : nullptr;
        if (a.perm_array && n > 0 && perm == nullptr) {
            if (threadIdx.x == 0) {
                a.out[k].logabsdet = NAN;
                a.out[k].sign = 0.0;
                a.out[k].info = MC_INFO_BADARG;
            }
            continue;
        }
        wg_factor<T>(static_cast<const T*>(a.A_array[k]), n, a.lda_array[k],
                     b, tile, a.update, region, a.out + k, sh, lds, perm);
    }
}

// ------------------------------------------------------------------ host

static std::atomic<bool> g_spare_xcc0{false};

int batched_spare_xcc0(int on) { return g_spare_xcc0.exchange(on != 0) ? 1 : 0; }
bool batched_spare_xcc0_on() { return g_spare_xcc0.load(); }

size_t batched_region_bytes(int64_t n_max, int dtype, const TuneTable& t,
                            bool with_w)
{
    const int elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    size_t best = 0;
    for (int k = 0; k < kTuneBuckets; ++k)
        best = std::max(best, bat_region_bytes(n_max, t.b[k], elem, with_w));
    return best;
}

size_t batched_lds_bytes(int dtype, const TuneTable& t)
{
    const int elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    int64_t bmax = 16;
    for (int k = 0; k < kTuneBuckets; ++k) bmax = std::max<int64_t>(bmax, t.b[k]);
    const int64_t nblk = (bmax + 15) / 16; // U11's upper and inverted diagonal blocks
    const size_t trsm = (size_t)elem * (size_t)(nblk * (nblk - 1) / 2 + nblk) * 256 +
                        sizeof(int) * 16 * (size_t)nblk;
    const size_t gemm = (size_t)elem * 2 * 16 * ((128 + 16) + (64 + 16)); // A and B, two buffers
    const size_t bf16 = 4 * 64 * (32 + 8) * 2;
    return std::max(trsm, std::max(gemm, bf16));
}

hipError_t launch_batched(const BatchArgs& a, int dtype, size_t lds_bytes,
                          hipStream_t stream)
{
    hipLaunchKernelGGL(batched_setup, dim3(1), dim3(kBT), 0, stream,
                       a.n_array, a.batch, a.counter, a.order);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return note_hip_error(e);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return note_hip_error(e);
    const int64_t grid = std::min<int64_t>((int64_t)cus * 2, std::max<int64_t>(a.batch, 1));
    // dynamic LDS above the 64 KB default needs the attribute raised to the
    // exact size (static LDS of the kernel adds to it within 160 KB)
    if (dtype == MC_DTYPE_F64) {
        if (lds_bytes > 64 * 1024) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batched_persistent<double>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e != hipSuccess) return note_hip_error(e);
        }
        hipLaunchKernelGGL(batched_persistent<double>, dim3((unsigned)grid), dim3(kBT),
                           lds_bytes, stream, a);
    } else {
        if (lds_bytes > 64 * 1024) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&batched_persistent<float>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e != hipSuccess) return note_hip_error(e);
        }
        hipLaunchKernelGGL(batched_persistent<float>, dim3((unsigned)grid), dim3(kBT),
                           lds_bytes, stream, a);
    }
    return note_hip_error(hipGetLastError());
}

} // namespace mc
