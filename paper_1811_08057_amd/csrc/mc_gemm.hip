// mc_gemm.hip -- MFMA kernels for the blocked path's trailing update.
//
// Block tile BT x BT of C (128 x 128, or 64 x 64 once too few tiles remain),
// a grid of wavefronts each owning a few 16 x 16 tiles.  -L and U stream
// through LDS in K chunks into accumulators that start from zero; the old C
// (read through colsrc, in the K loop or the epilogue) is added and the
// result stored in place.  Per block: 2 * BT^2 * K flops against
// BT^2 * 2 * sizeof(T) bytes of C traffic, so the update is matrix-core
// bound once K = b is large enough (b/8 flop per byte in FP64).  Three
// launch forms: a tile per block (`gemm_scalar`, `gemm_bf16x3`); beside a
// panel chain, a resident wave of blocks taking tiles from a counter off
// XCD 0 (`*_spare`); and the next panel's rows, every operand staged at
// once (`gemm_rows`).
//
// Operand and accumulator layouts: mc_mfma.h.
#include "mc_gemm.h"
#include "mc_device.h"
#include "mc_mfma.h"

#include <algorithm>

namespace mc {


// The trailing update comes in two forms, one kernel each (a single kernel
// with both keeps more registers live and spills):
// - one tile per block, at blockIdx (a two-dimensional grid);
// - beside a panel chain on XCD 0 (tile_ctr set): one resident wave of
//   blocks, 8 W of them for W blocks resident per XCD.  Workgroups go to
//   the XCDs in turn, so each XCD receives W.  Those on XCD 0 leave before
//   any memory access (workgroups are dispatched in order: while one of
//   them waits for a compute unit there, the other XCDs' blocks wait too);
//   the others take tiles from the counter, in row-major order.  Which
//   blocks those are does not matter for the result.
// The tile loop: thread 0 asks for the next tile while the block works on
// the current one.  The last barrier of a tile's K loop follows its last
// LDS read, so the next tile may refill the buffers at once.
template <typename T, class F>
__device__ __forceinline__ void counter_tiles(const GemmArgs<T>& g, int bm, int bn,
                                              F&& tile)
{
    __shared__ unsigned int sh_t;
    const int64_t ntx = (g.N + bn - 1) / bn, tiles = ntx * ((g.M + bm - 1) / bm);
    if (threadIdx.x == 0) sh_t = atomicAdd(g.tile_ctr, 1u);
    __syncthreads();
    int64_t t = sh_t;
    while (t < tiles) {
        unsigned int nt = 0;
        if (threadIdx.x == 0) nt = atomicAdd(g.tile_ctr, 1u);
        const int64_t ty = t / ntx;
        tile(ty * bm, (t - ty * ntx) * bn);
        if (threadIdx.x == 0) sh_t = nt;
        __syncthreads();
        t = sh_t;
    }
}

// ---------------------------------------------------------------------------
// FP64 / FP32: one scalar operand per lane, K = 4 per instruction.  The
// block is WGM x WGN wavefronts, each owning TM x TN tiles of 16 x 16.  The
// K loop is double-buffered: chunk c+1 is read from global memory into
// registers while chunk c feeds the matrix cores, then parked in the other
// LDS buffer; one barrier per chunk.  The matrix cores need several
// wavefronts issuing per SIMD; the FP64 128 x 128 tile uses 16 wavefronts
// of 32 x 32 (four per SIMD, 128 VGPRs each), small enough per wavefront to
// also hold the tile's old C, read inside the K loop (PF) so that the
// epilogue waits on no load: 32.4 against 29.4 TFLOP/s for 8 wavefronts of
// 64 x 32 with C read in the epilogue (M = 7744, N = 7872, K = 128), and
// 27.4 against 22.9 on the seven XCDs beside a panel chain.  In FP32 the
// same 16 wavefronts fit twice per compute unit without C (49 VGPRs), which
// is faster still: 65.7 against 56.0 TFLOP/s with C and 51.2 for 8.
template <class P, int WGM, int WGN, int TM, int TN, bool PF, int KC = 16>
__device__ __forceinline__ void scalar_tile(const GemmArgs<typename P::T>& g,
                                            int64_t rb, int64_t cb, int tid)
{
    using T = typename P::T;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int BM = 16 * TM * WGM, BN = 16 * TN * WGN;
    constexpr int LDA = BM + 16, LDB = BN + 16; // conflict-free fragment reads
    constexpr int PA = (BM * KC + NT - 1) / NT, PB = (BN * KC + NT - 1) / NT;
    __shared__ T As[2][KC][LDA]; // -L, transposed (k major)
    __shared__ T Bs[2][KC][LDB]; // U

    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wid / WGN, wn = wid % WGN;
    const int col_in = lane & 15, kq_lane = lane >> 4;

    T pa[PA], pb[PB];
    // L's rows rb.. (rows past M lie past the range) and U's K rows from
    // column c0 + cb
    const __amdgpu_buffer_rsrc_t rl = operand_rsrc(
        g.L + rb * g.ldl, sizeof(T) * std::min<int64_t>(BM, g.M - rb) * g.ldl);
    const __amdgpu_buffer_rsrc_t ru = operand_rsrc(
        g.U + g.c0 + cb, sizeof(T) * ((int64_t)(g.K - 1) * g.ldu + (g.N - cb)));
    auto gload = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int e = tid + p * NT;
            const int rr = e / KC, kk = e - rr * KC;
            const bool ok = e < BM * KC && k0 + kk < g.K;
            pa[p] = operand_load<T>(
                rl, ok ? (uint32_t)(sizeof(T) * (rr * g.ldl + k0 + kk)) : kOutOfRange);
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int e = tid + p * NT;
            const int kb = e / BN, cc = e - kb * BN;
            const bool ok = e < BN * KC && cb + cc < g.N && k0 + kb < g.K;
            pb[p] = operand_load<T>(
                ru, ok ? (uint32_t)(sizeof(T) * ((int64_t)(k0 + kb) * g.ldu + cc)) : kOutOfRange);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int e = tid + p * NT;
            const int rr = e / KC, kk = e - rr * KC;
            if (e < BM * KC) As[buf][kk][rr] = -pa[p];
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int e = tid + p * NT;
            const int kb = e / BN, cc = e - kb * BN;
            if (e < BN * KC) Bs[buf][kb][cc] = pb[p];
        }
    };

    // PF: the sources of this wavefront's columns, read first so that no
    // later wait is for them alone
    int csrc[TN];
    if (PF) {
        const __amdgpu_buffer_rsrc_t rc =
            operand_rsrc(g.colsrc + g.c0 + cb, sizeof(int) * (g.N - cb));
#pragma unroll
        for (int tj = 0; tj < TN; ++tj) {
            const int cc = wn * 16 * TN + tj * 16 + col_in;
            csrc[tj] = (int)__builtin_amdgcn_raw_buffer_load_b32(
                rc, cb + cc < g.N ? (uint32_t)(sizeof(int) * cc) : kOutOfRange, 0, 0);
        }
    }
    gload(0);

    // the product -L U accumulates from zero; C joins it in the epilogue, so
    // the K loop holds only accumulators, operands and the prefetch
    typename P::Acc acc[TM][TN];
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TN; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[ti][tj][r] = T(0);

    sstore(0);
    __syncthreads();
    const int nch = (g.K + KC - 1) / KC;
    T cpre[TM][TN][4]; // PF: the tile's old C
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload((c + 1) * KC);
        if (PF && c == 0) {
            // the old C, read behind the next chunk's operands: loads
            // complete in order, so no wait before the chunk after that
            // includes these, and by then they are in
            const __amdgpu_buffer_rsrc_t rcm = operand_rsrc(
                g.C + (g.r0 + rb) * g.ldc, sizeof(T) * std::min<int64_t>(BM, g.M - rb) * g.ldc);
#pragma unroll
            for (int tj = 0; tj < TN; ++tj) {
                const bool okc = cb + wn * 16 * TN + tj * 16 + col_in < g.N;
#pragma unroll
                for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rr = wm * 16 * TM + ti * 16 + P::drow(lane, r);
                        cpre[ti][tj][r] = operand_load<T>(
                            rcm, okc ? (uint32_t)(sizeof(T) * (rr * g.ldc + csrc[tj]))
                                     : kOutOfRange);
                    }
            }
        }
#pragma unroll
        for (int kq = 0; kq < KC; kq += 4) {
            T a[TM], b[TN];
#pragma unroll
            for (int t = 0; t < TM; ++t)
                a[t] = As[buf][kq + kq_lane][wm * 16 * TM + t * 16 + col_in];
#pragma unroll
            for (int t = 0; t < TN; ++t)
                b[t] = Bs[buf][kq + kq_lane][wn * 16 * TN + t * 16 + col_in];
#pragma unroll
            for (int ti = 0; ti < TM; ++ti)
#pragma unroll
                for (int tj = 0; tj < TN; ++tj)
                    acc[ti][tj] = P::mma(a[ti], b[tj], acc[ti][tj]);
        }
        if (c + 1 < nch) sstore(buf ^ 1);
        __syncthreads();
    }

    // C[dst] = C[src] + acc.  A moved column's source lies in the panel's
    // column range, which no block writes; otherwise src == dst and the
    // same thread reads before it writes.
#pragma unroll
    for (int tj = 0; tj < TN; ++tj) {
        const int64_t col = cb + wn * 16 * TN + tj * 16 + col_in;
        if (col >= g.N) continue;
        const int64_t src = g.colsrc[g.c0 + col];
#pragma unroll
        for (int ti = 0; ti < TM; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = rb + wm * 16 * TM + ti * 16 + P::drow(lane, r);
                if (row < g.M) {
                    T* crow = g.C + (g.r0 + row) * g.ldc;
                    crow[g.c0 + col] = (PF ? cpre[ti][tj][r] : crow[src]) + acc[ti][tj][r];
                }
            }
    }
}

// The last barrier of a tile's K loop follows its last LDS read, so the
// next tile may refill the buffers at once.
// WPS: wavefronts per SIMD the launch bound asks for (the register budget:
// 512 / WPS VGPRs); PF: the old C read inside the K loop.
template <class P, int WGM, int WGN, int TM, int TN, int WPS, bool PF, int KC = 16>
__global__ void __launch_bounds__(64 * WGM * WGN, WPS)
gemm_scalar(GemmArgs<typename P::T> g)
{
    if (g.state->status != kStatusOk) return;
    constexpr int BM = 16 * TM * WGM, BN = 16 * TN * WGN;
    scalar_tile<P, WGM, WGN, TM, TN, PF, KC>(g, (int64_t)blockIdx.y * BM,
                                             (int64_t)blockIdx.x * BN, (int)threadIdx.x);
}

template <class P, int WGM, int WGN, int TM, int TN, int WPS, bool PF, int KC = 16>
__global__ void __launch_bounds__(64 * WGM * WGN, WPS)
gemm_scalar_spare(GemmArgs<typename P::T> g)
{
    if (xcc_id() == 0) return; // the panel chain's XCD: no memory access
    if (g.state->status != kStatusOk) return;
    constexpr int BM = 16 * TM * WGM, BN = 16 * TN * WGN;
    counter_tiles(g, BM, BN, [&](int64_t rb, int64_t cb) {
        // formed afresh per tile: kept across the tile loop, the addresses
        // derived from it would hold registers through the K loop
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        scalar_tile<P, WGM, WGN, TM, TN, PF, KC>(g, rb, cb, tid);
    });
}

// ---------------------------------------------------------------------------
// Split-BF16 x 3 with FP32 accumulation: x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even), and
//     a b ~= a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo term is ~2^-16 relative).  K = 32 per instruction.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// WG x WG wavefronts, each owning WT x WT tiles of 16 x 16 (block tile
// 16 WT WG).
template <int WT, int WG>
__device__ __forceinline__ void bf16x3_tile(const GemmArgs<float>& g, int64_t rb,
                                            int64_t cb, int tid)
{
    constexpr int BT = 16 * WT * WG, NT = 64 * WG * WG;
    constexpr int KC = 32;
    constexpr int LD = KC + 8; // bf16 elements per LDS row (16-byte aligned)
    constexpr int PA = (BT * KC + NT - 1) / NT;
    // two buffers: chunk c+1 is read into registers while chunk c feeds the
    // matrix cores, then split and parked in the other buffer
    __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BT][LD], Al[2][BT][LD];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BT][LD], Bl[2][BT][LD];

    const int lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wid / WG, wn = wid % WG;
    const int col_in = lane & 15, kg = lane >> 4;

    const __amdgpu_buffer_rsrc_t rl = operand_rsrc(
        g.L + rb * g.ldl, sizeof(float) * std::min<int64_t>(BT, g.M - rb) * g.ldl);
    const __amdgpu_buffer_rsrc_t ru = operand_rsrc(
        g.U + g.c0 + cb, sizeof(float) * ((int64_t)(g.K - 1) * g.ldu + (g.N - cb)));
    float pa[PA], pb[PA];
    auto gload = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int e = tid + p * NT;
            { // A = -L: row-major in global and in LDS (k contiguous)
                const int rr = e / KC, kk = e - rr * KC;
                const bool ok = e < BT * KC && k0 + kk < g.K;
                pa[p] = operand_load<float>(
                    rl, ok ? (uint32_t)(sizeof(float) * (rr * g.ldl + k0 + kk)) : kOutOfRange);
            }
            { // B = U: k-major in global, stored column-major (k contiguous)
                const int kk = e / BT, cc = e - kk * BT;
                const bool ok = e < BT * KC && cb + cc < g.N && k0 + kk < g.K;
                pb[p] = operand_load<float>(
                    ru, ok ? (uint32_t)(sizeof(float) * ((int64_t)(k0 + kk) * g.ldu + cc))
                           : kOutOfRange);
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int e = tid + p * NT;
            if (e < BT * KC) {
                const int rr = e / KC, kk = e - rr * KC;
                split_bf16(-pa[p], Ah[buf][rr][kk], Al[buf][rr][kk]);
                const int kb = e / BT, cc = e - kb * BT;
                split_bf16(pb[p], Bh[buf][cc][kb], Bl[buf][cc][kb]);
            }
        }
    };

    // the sources of this wavefront's columns, then the first chunk
    int csrc[WT];
    {
        const __amdgpu_buffer_rsrc_t rc =
            operand_rsrc(g.colsrc + g.c0 + cb, sizeof(int) * (g.N - cb));
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) {
            const int cc = wn * 16 * WT + tj * 16 + col_in;
            csrc[tj] = (int)__builtin_amdgcn_raw_buffer_load_b32(
                rc, cb + cc < g.N ? (uint32_t)(sizeof(int) * cc) : kOutOfRange, 0, 0);
        }
    }
    gload(0);

    f4 acc[WT][WT];
#pragma unroll
    for (int ti = 0; ti < WT; ++ti)
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) acc[ti][tj] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    sstore(0);
    __syncthreads();
    const int nch = (g.K + KC - 1) / KC;
    float cpre[WT][WT][4]; // the tile's old C, read behind chunk 1's operands
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload((c + 1) * KC);
        if (c == 0) {
            const __amdgpu_buffer_rsrc_t rcm = operand_rsrc(
                g.C + (g.r0 + rb) * g.ldc,
                sizeof(float) * std::min<int64_t>(BT, g.M - rb) * g.ldc);
#pragma unroll
            for (int tj = 0; tj < WT; ++tj) {
                const bool okc = cb + wn * 16 * WT + tj * 16 + col_in < g.N;
#pragma unroll
                for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rr = wm * 16 * WT + ti * 16 + 4 * kg + r;
                        cpre[ti][tj][r] = operand_load<float>(
                            rcm, okc ? (uint32_t)(sizeof(float) * (rr * g.ldc + csrc[tj]))
                                     : kOutOfRange);
                    }
            }
        }
        bf8 ah[WT], al[WT], bh[WT], bl[WT];
#pragma unroll
        for (int t = 0; t < WT; ++t) {
            const int ar = wm * 16 * WT + t * 16 + col_in;
            const int bc = wn * 16 * WT + t * 16 + col_in;
            ah[t] = *reinterpret_cast<const bf8*>(&Ah[buf][ar][8 * kg]);
            al[t] = *reinterpret_cast<const bf8*>(&Al[buf][ar][8 * kg]);
            bh[t] = *reinterpret_cast<const bf8*>(&Bh[buf][bc][8 * kg]);
            bl[t] = *reinterpret_cast<const bf8*>(&Bl[buf][bc][8 * kg]);
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
        if (c + 1 < nch) sstore(buf ^ 1);
        __syncthreads();
    }

    // C[dst] = C[src] + acc.  A moved column's source lies in the panel's
    // column range, which no block writes.
#pragma unroll
    for (int tj = 0; tj < WT; ++tj) {
        const int64_t col = cb + wn * 16 * WT + tj * 16 + col_in;
        if (col >= g.N) continue;
#pragma unroll
        for (int ti = 0; ti < WT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = rb + wm * 16 * WT + ti * 16 + 4 * kg + r;
                if (row < g.M)
                    g.C[(g.r0 + row) * g.ldc + g.c0 + col] = cpre[ti][tj][r] + acc[ti][tj][r];
            }
    }
}

template <int WT, int WG>
__global__ void __launch_bounds__(64 * WG * WG)
gemm_bf16x3(GemmArgs<float> g)
{
    if (g.state->status != kStatusOk) return;
    constexpr int BT = 16 * WT * WG;
    bf16x3_tile<WT, WG>(g, (int64_t)blockIdx.y * BT, (int64_t)blockIdx.x * BT,
                        (int)threadIdx.x);
}

template <int WT, int WG>
__global__ void __launch_bounds__(64 * WG * WG)
gemm_bf16x3_spare(GemmArgs<float> g)
{
    if (xcc_id() == 0) return; // the panel chain's XCD: no memory access
    if (g.state->status != kStatusOk) return;
    constexpr int BT = 16 * WT * WG;
    counter_tiles(g, BT, BT, [&](int64_t rb, int64_t cb) {
        int tid = (int)threadIdx.x; // formed afresh per tile (as gemm_scalar_spare)
        asm volatile("" : "+v"(tid));
        bf16x3_tile<WT, WG>(g, rb, cb, tid);
    });
}

// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Updates of 65..128 rows (the next panel's rows),
// FP64 or FP32 operands, K <= kMaxPanel.  Too few tiles to hide latency
// behind other blocks, so a block keeps everything in flight at once:
// - its whole K of -L and U goes to LDS from one round of 16-byte loads,
//   issued with the reads of the old C (through colsrc);
// - each of the four wavefronts takes a quarter of K for the whole 64 x 64
//   tile (16 independent accumulators, chains of K/16 products, where one
//   wavefront per 32 x 32 quarter would chain K/4 dependent products);
// - the four partial tiles are summed through LDS, each wavefront then
//   finishing 16 rows.
// One block per compute unit.
template <class P>
__global__ void __launch_bounds__(256, 1)
gemm_rows(GemmArgs<typename P::T> g)
{
    using T = typename P::T;
    constexpr int BT = 64, KM = (int)kMaxPanel;
    constexpr int LD = BT + (sizeof(T) == 8 ? 8 : 16); // U's row pitch
    constexpr int LK = KM + 4;                          // -L's row pitch
    constexpr int V = 16 / sizeof(T);                   // elements per 16 bytes
    constexpr int PE = BT * KM / (256 * V);             // 16-byte loads per tile
    constexpr int RL = BT + (sizeof(T) == 8 ? 2 : 4);   // partial-tile row pitch
    constexpr int NL = BT * LK + KM * LD;               // both tiles, within 160 KB
    static_assert(4 * BT * RL <= NL, "partials fit in the operand space");
    __shared__ T lds[NL];
    // -L row major (a row's K entries contiguous, so a wavefront's 16-byte
    // stores cover whole rows; the pad spreads the fragment reads, 16 rows
    // by 4 k, over the banks), U k major
    T (*As)[LK] = reinterpret_cast<T (*)[LK]>(lds);
    T (*Bs)[LD] = reinterpret_cast<T (*)[LD]>(lds + BT * LK);
    if (g.state->status != kStatusOk) return;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col_in = lane & 15;
    const int64_t rb = (int64_t)blockIdx.y * BT, cb = (int64_t)blockIdx.x * BT;
    const int K = g.K;
    typedef T tv __attribute__((ext_vector_type(V)));

    // Every load goes through a buffer descriptor, entries outside an
    // operand at an offset past its range (read as zero), so none sits in a
    // branch and all of them are in flight together.
    // The finishing rows of this thread: row fr + 4 q (q = 0..3) of its
    // wavefront's 16, column fc.
    const int fr = wid * 16 + (lane >> 4), fc = (lane & 15) * 4;
    const __amdgpu_buffer_rsrc_t rl =
        operand_rsrc(g.L, (int64_t)sizeof(T) * ((g.M - 1) * g.ldl + K));
    const __amdgpu_buffer_rsrc_t ru =
        operand_rsrc(g.U + g.c0, (int64_t)sizeof(T) * ((int64_t)(K - 1) * g.ldu + g.N));
    // 16-byte loads where every vector lies wholly inside or wholly outside
    // its operand and the rows are 16-byte aligned (the blocked path's L and
    // W are; a caller's matrix need not be): the same for the whole block
    const bool vec = K % V == 0 && cb + BT <= g.N &&
                     ((reinterpret_cast<uintptr_t>(g.L) | (uintptr_t)g.ldl * sizeof(T)) & 15) == 0 &&
                     ((reinterpret_cast<uintptr_t>(g.U + g.c0) | (uintptr_t)g.ldu * sizeof(T)) &
                      15) == 0;
    tv pa[PE], pb[PE];
    if (vec) {
#pragma unroll
        for (int p = 0; p < PE; ++p) {
            const int e = (tid + 256 * p) * V;
            const int rr = e / KM, kk = e % KM; // L: rows of K contiguous
            const int64_t row = rb + rr;
            const uint32_t lo = row < g.M && kk < K
                                    ? (uint32_t)(sizeof(T) * (row * g.ldl + kk))
                                    : kOutOfRange;
            pa[p] = __builtin_bit_cast(tv, __builtin_amdgcn_raw_buffer_load_b128(rl, lo, 0, 0));
            const int kb = e / BT, cc = e % BT; // U: K rows of 64 columns
            const uint32_t uo = kb < K ? (uint32_t)(sizeof(T) * ((int64_t)kb * g.ldu + cb + cc))
                                       : kOutOfRange;
            pb[p] = __builtin_bit_cast(tv, __builtin_amdgcn_raw_buffer_load_b128(ru, uo, 0, 0));
        }
    } else {
#pragma unroll
        for (int p = 0; p < PE; ++p) {
            const int e = (tid + 256 * p) * V;
            const int rr = e / KM, kk = e % KM;
            const int64_t row = rb + rr;
            const int kb = e / BT, cc = e % BT;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const uint32_t lo = row < g.M && kk + v < K
                                        ? (uint32_t)(sizeof(T) * (row * g.ldl + kk + v))
                                        : kOutOfRange;
                pa[p][v] = operand_load<T>(rl, lo);
                const int64_t col = cb + cc + v;
                const uint32_t uo = kb < K && col < g.N
                                        ? (uint32_t)(sizeof(T) * ((int64_t)kb * g.ldu + col))
                                        : kOutOfRange;
                pb[p][v] = operand_load<T>(ru, uo);
            }
        }
    }
    const __amdgpu_buffer_rsrc_t rcs = operand_rsrc(g.colsrc + g.c0, sizeof(int) * g.N);
    int src[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t col = cb + fc + q;
        src[q] = (int)__builtin_amdgcn_raw_buffer_load_b32(
            rcs, col < g.N ? (uint32_t)(sizeof(int) * col) : kOutOfRange, 0, 0);
    }
    // the old C through colsrc (rows past M and columns past N read zero)
    const __amdgpu_buffer_rsrc_t rc =
        operand_rsrc(g.C + g.r0 * g.ldc, (int64_t)sizeof(T) * g.M * g.ldc);
    T cold[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = rb + fr + 4 * r;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            cold[r][q] = operand_load<T>(
                rc, row < g.M && cb + fc + q < g.N
                        ? (uint32_t)(sizeof(T) * (row * g.ldc + src[q]))
                        : kOutOfRange);
    }
#pragma unroll
    for (int p = 0; p < PE; ++p) {
        const int e = (tid + 256 * p) * V;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            As[(e + v) / KM][(e + v) % KM] = -pa[p][v];
            Bs[(e + v) / BT][(e + v) % BT] = pb[p][v];
        }
    }
    __syncthreads();

    // this wavefront's quarter of K (entries past K are zero)
    typename P::Acc acc[4][4];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[ti][tj][r] = T(0);
    const int kq_lane = lane >> 4, kspan = ((K + 15) / 16) * 4;
    const int k0 = wid * kspan, k1 = k0 + kspan;
    for (int kq = k0; kq < k1; kq += 4) {
        T a[4], b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[t] = As[t * 16 + col_in][kq + kq_lane];
            b[t] = Bs[kq + kq_lane][t * 16 + col_in];
        }
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
            for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = P::mma(a[ti], b[tj], acc[ti][tj]);
    }
    __syncthreads(); // the operands are no longer read: partials go there
    T* part = lds + wid * BT * RL;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[(ti * 16 + P::drow(lane, r)) * RL + tj * 16 + col_in] = acc[ti][tj][r];
    __syncthreads();

    // C[dst] = C[src] + the four partials (a moved column's source lies in
    // the panel's column range, which no block writes; src == dst otherwise)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = rb + fr + 4 * r;
        if (row >= g.M) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t col = cb + fc + q;
            if (col >= g.N) continue;
            const int o = (fr + 4 * r) * RL + fc + q;
            T v = cold[r][q];
#pragma unroll
            for (int w4 = 0; w4 < 4; ++w4) v += lds[w4 * BT * RL + o];
            g.C[(g.r0 + row) * g.ldc + g.c0 + col] = v;
        }
    }
}

// Large tiles while they still give every CU work; smaller ones after.
static bool big_tiles(int64_t M, int64_t N)
{
    return ((M + 127) / 128) * ((N + 127) / 128) >= 512;
}

// gemm_rows: 65..128 rows (the next panel's) and K <= kMaxPanel, not beside
// a panel chain.  (Measured at N = 7867, K = 128: 22.0 against 24.7 us for
// 128 rows with gemm_scalar's 64 x 64 tiles; below 64 rows gemm_scalar is
// the faster, 17.5 against 20.3 us at 37 rows.)
template <typename T>
static bool rows_form(const GemmArgs<T>& g)
{
    return !g.tile_ctr && g.M > 64 && g.M <= 128 && g.K <= kMaxPanel;
}

// Blocks of kernel k resident on one XCD at a time (compute units per XCD
// times blocks per compute unit); at least 1.
template <class Kern>
static int64_t blocks_per_xcd(Kern k, int threads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k),
                                                     threads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 64;
    }
    return std::max<int64_t>(1, (int64_t)(cus / 8) * per_cu);
}

// The update's launch: kernel `one` (a tile per block) on a two-dimensional
// grid, or `spare` (the form beside a panel chain) on one resident wave of
// blocks, no more than the tiles need.
template <class Kern, class Args>
static void launch_grid(Kern one, Kern spare, const Args& g, int bm, int bn,
                        int threads, hipStream_t stream)
{
    const int64_t tx = (g.N + bn - 1) / bn, ty = (g.M + bm - 1) / bm;
    if (g.tile_ctr) {
        const int64_t groups = std::min<int64_t>(blocks_per_xcd(spare, threads),
                                                 (tx * ty + 6) / 7);
        hipLaunchKernelGGL(spare, dim3((unsigned)(8 * groups)), dim3(threads), 0,
                           stream, g);
    } else {
        hipLaunchKernelGGL(one, dim3((unsigned)tx, (unsigned)ty), dim3(threads), 0,
                           stream, g);
    }
}

template <>
hipError_t launch_trailing_update<double>(const GemmArgs<double>& g,
                                          int update, hipStream_t stream)
{
    if (update != MC_UPDATE_NATIVE) return hipErrorInvalidValue;
    if (rows_form(g)) {
        hipLaunchKernelGGL(gemm_rows<MfmaF64>, dim3((unsigned)((g.N + 63) / 64),
                                                    (unsigned)((g.M + 63) / 64)),
                           dim3(256), 0, stream, g);
        return hipGetLastError();
    }
    if (big_tiles(g.M, g.N)) // 16 waves (4 x 4), 32 x 32 per wave: 128 x 128,
        // four waves per SIMD with room for the old C (read in the K loop)
        launch_grid(gemm_scalar<MfmaF64, 4, 4, 2, 2, 4, true>,
                    gemm_scalar_spare<MfmaF64, 4, 4, 2, 2, 4, true>, g, 128, 128, 1024, stream);
    else // 4 waves (2 x 2), 32 x 32 per wave: 64 x 64
        launch_grid(gemm_scalar<MfmaF64, 2, 2, 2, 2, 2, false>,
                    gemm_scalar_spare<MfmaF64, 2, 2, 2, 2, 2, false>, g, 64, 64, 256, stream);
    return hipGetLastError();
}

template <>
hipError_t launch_trailing_update<float>(const GemmArgs<float>& g, int update,
                                         hipStream_t stream)
{
    const bool big = big_tiles(g.M, g.N);
    if (update == MC_UPDATE_BF16X3) {
        if (big)
            // 16 waves of 32 x 32: 74.1 against 41.2 TFLOP/s for 4 of 64 x 64
            // (M = 7744, N = 7872, K = 128)
            launch_grid(gemm_bf16x3<2, 4>, gemm_bf16x3_spare<2, 4>, g, 128, 128, 1024, stream);
        else
            launch_grid(gemm_bf16x3<2, 2>, gemm_bf16x3_spare<2, 2>, g, 64, 64, 256, stream);
    } else if (rows_form(g)) {
        hipLaunchKernelGGL(gemm_rows<MfmaF32>, dim3((unsigned)((g.N + 63) / 64),
                                                    (unsigned)((g.M + 63) / 64)),
                           dim3(256), 0, stream, g);
    } else {
        if (big) // 16 waves of 32 x 32, two blocks per compute unit
            launch_grid(gemm_scalar<MfmaF32, 4, 4, 2, 2, 4, false>,
                        gemm_scalar_spare<MfmaF32, 4, 4, 2, 2, 4, false>, g, 128, 128, 1024,
                        stream);
        else
            launch_grid(gemm_scalar<MfmaF32, 2, 2, 2, 2, 2, false>,
                        gemm_scalar_spare<MfmaF32, 2, 2, 2, 2, 2, false>, g, 64, 64, 256,
                        stream);
    }
    return hipGetLastError();
}

} // namespace mc
