// mc_gemm.hip -- MFMA kernels for the blocked path's trailing update.
//
// Block tile BT x BT of C (BT = 32 * WT), four wavefronts in a 2 x 2 grid,
// each owning WT x WT tiles of 16 x 16.  -L and U stream through LDS in K
// chunks into accumulators that start from zero; the epilogue adds the old
// C (read through colsrc) and stores in place.  Per block: 2 * BT^2 * K
// flops against BT^2 * 2 * sizeof(T) bytes of C traffic, so the update is
// matrix-core bound once K = b is large enough (b/8 flop per byte in FP64).
//
// Operand and accumulator layouts: mc_mfma.h.
#include "mc_gemm.h"
#include "mc_device.h"
#include "mc_mfma.h"

#include <algorithm>

namespace mc {

constexpr int kGemmThreads = 256;

// ---------------------------------------------------------------------------
// FP64 / FP32: one scalar operand per lane, K = 4 per instruction.  The
// K loop is double-buffered: chunk c+1 is read from global memory into
// registers while chunk c feeds the matrix cores, then parked in the other
// LDS buffer; one barrier per chunk.
// (two blocks per CU: the register budget then covers the 64 FP64
// accumulators of a 4 x 4 wave tile without spilling)
template <class P, int WT>
__global__ void __launch_bounds__(kGemmThreads, 2)
gemm_scalar(GemmArgs<typename P::T> g)
{
    using T = typename P::T;
    constexpr int BT = 32 * WT;
    constexpr int KC = 16;
    constexpr int LDS_LD = BT + 16;               // conflict-free fragment reads
    constexpr int PE = BT * KC / kGemmThreads;    // elements per thread per chunk
    __shared__ T As[2][KC][LDS_LD];               // -L, transposed (k major)
    __shared__ T Bs[2][KC][LDS_LD];               // U
    if (g.state->status != kStatusOk) return;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int64_t rb = (int64_t)blockIdx.y * BT, cb = (int64_t)blockIdx.x * BT;
    const int col_in = lane & 15, kq_lane = lane >> 4;

    T pa[PE], pb[PE];
    auto gload = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PE; ++p) {
            const int e = tid + p * kGemmThreads;
            const int rr = e / KC, kk = e - rr * KC;
            const int64_t row = rb + rr;
            pa[p] = (row < g.M && k0 + kk < g.K) ? -g.L[row * g.ldl + k0 + kk]
                                                 : T(0);
            const int kb = e / BT, cc = e - kb * BT;
            const int64_t col = cb + cc;
            pb[p] = (col < g.N && k0 + kb < g.K)
                        ? g.U[(int64_t)(k0 + kb) * g.ldu + g.c0 + col]
                        : T(0);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PE; ++p) {
            const int e = tid + p * kGemmThreads;
            const int rr = e / KC, kk = e - rr * KC;
            As[buf][kk][rr] = pa[p];
            const int kb = e / BT, cc = e - kb * BT;
            Bs[buf][kb][cc] = pb[p];
        }
    };

    gload(0);

    // the product -L U accumulates from zero; C joins it in the epilogue, so
    // the K loop holds only accumulators, operands and the prefetch
    typename P::Acc acc[WT][WT];
#pragma unroll
    for (int ti = 0; ti < WT; ++ti)
#pragma unroll
        for (int tj = 0; tj < WT; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[ti][tj][r] = T(0);

    sstore(0);
    __syncthreads();
    const int nch = (g.K + KC - 1) / KC;
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload((c + 1) * KC);
#pragma unroll
        for (int kq = 0; kq < KC; kq += 4) {
            T a[WT], b[WT];
#pragma unroll
            for (int t = 0; t < WT; ++t) {
                a[t] = As[buf][kq + kq_lane][wm * 16 * WT + t * 16 + col_in];
                b[t] = Bs[buf][kq + kq_lane][wn * 16 * WT + t * 16 + col_in];
            }
#pragma unroll
            for (int ti = 0; ti < WT; ++ti)
#pragma unroll
                for (int tj = 0; tj < WT; ++tj)
                    acc[ti][tj] = P::mma(a[ti], b[tj], acc[ti][tj]);
        }
        if (c + 1 < nch) sstore(buf ^ 1);
        __syncthreads();
    }

    // C[dst] = C[src] + acc.  A moved column's source lies in the panel's
    // column range, which no block writes; otherwise src == dst and the
    // same thread reads before it writes.
#pragma unroll
    for (int tj = 0; tj < WT; ++tj) {
        const int64_t col = cb + wn * 16 * WT + tj * 16 + col_in;
        if (col >= g.N) continue;
        const int64_t src = g.colsrc[g.c0 + col];
#pragma unroll
        for (int ti = 0; ti < WT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = rb + wm * 16 * WT + ti * 16 + P::drow(lane, r);
                if (row < g.M) {
                    T* crow = g.C + (g.r0 + row) * g.ldc;
                    crow[g.c0 + col] = crow[src] + acc[ti][tj][r];
                }
            }
    }
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

template <int WT>
__global__ void __launch_bounds__(kGemmThreads)
gemm_bf16x3(GemmArgs<float> g)
{
    constexpr int BT = 32 * WT;
    constexpr int KC = 32;
    constexpr int LD = KC + 8; // bf16 elements per LDS row (16-byte aligned)
    __shared__ __attribute__((aligned(16))) __bf16 Ah[BT][LD], Al[BT][LD];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[BT][LD], Bl[BT][LD];
    if (g.state->status != kStatusOk) return;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int64_t rb = (int64_t)blockIdx.y * BT, cb = (int64_t)blockIdx.x * BT;
    const int col_in = lane & 15, kg = lane >> 4;

    f4 acc[WT][WT];
#pragma unroll
    for (int ti = 0; ti < WT; ++ti)
#pragma unroll
        for (int tj = 0; tj < WT; ++tj) acc[ti][tj] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < g.K; k0 += KC) {
        // A = -L: row-major in global and in LDS (k contiguous)
        for (int e = tid; e < BT * KC; e += kGemmThreads) {
            const int rr = e / KC, kk = e - rr * KC;
            const int64_t row = rb + rr;
            const float v = (row < g.M && k0 + kk < g.K)
                                ? -g.L[row * g.ldl + k0 + kk]
                                : 0.0f;
            split_bf16(v, Ah[rr][kk], Al[rr][kk]);
        }
        // B = U: k-major in global, stored column-major (k contiguous)
        for (int e = tid; e < BT * KC; e += kGemmThreads) {
            const int kk = e / BT, cc = e - kk * BT;
            const int64_t col = cb + cc;
            const float v = (col < g.N && k0 + kk < g.K)
                                ? g.U[(int64_t)(k0 + kk) * g.ldu + g.c0 + col]
                                : 0.0f;
            split_bf16(v, Bh[cc][kk], Bl[cc][kk]);
        }
        __syncthreads();
        bf8 ah[WT], al[WT], bh[WT], bl[WT];
#pragma unroll
        for (int t = 0; t < WT; ++t) {
            const int ar = wm * 16 * WT + t * 16 + col_in;
            const int bc = wn * 16 * WT + t * 16 + col_in;
            ah[t] = *reinterpret_cast<const bf8*>(&Ah[ar][8 * kg]);
            al[t] = *reinterpret_cast<const bf8*>(&Al[ar][8 * kg]);
            bh[t] = *reinterpret_cast<const bf8*>(&Bh[bc][8 * kg]);
            bl[t] = *reinterpret_cast<const bf8*>(&Bl[bc][8 * kg]);
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
        const int64_t col = cb + wn * 16 * WT + tj * 16 + col_in;
        if (col >= g.N) continue;
        const int64_t src = g.colsrc[g.c0 + col];
#pragma unroll
        for (int ti = 0; ti < WT; ++ti)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = rb + wm * 16 * WT + ti * 16 + 4 * kg + r;
                if (row < g.M) {
                    float* crow = g.C + (g.r0 + row) * g.ldc;
                    crow[g.c0 + col] = crow[src] + acc[ti][tj][r];
                }
            }
    }
}

// ---------------------------------------------------------------------------

// Large tiles while they still give every CU work; smaller ones after.
static int pick_wt(int64_t M, int64_t N)
{
    const int64_t big = ((M + 127) / 128) * ((N + 127) / 128);
    return big >= 512 ? 4 : 2;
}

template <int WT, class Kern, class Args>
static void launch_tiles(Kern k, const Args& g, hipStream_t stream)
{
    constexpr int BT = 32 * WT;
    const dim3 grid((unsigned)((g.N + BT - 1) / BT),
                    (unsigned)((g.M + BT - 1) / BT));
    hipLaunchKernelGGL(k, grid, dim3(kGemmThreads), 0, stream, g);
}

template <>
hipError_t launch_trailing_update<double>(const GemmArgs<double>& g,
                                          int update, hipStream_t stream)
{
    if (update != MC_UPDATE_NATIVE) return hipErrorInvalidValue;
    if (pick_wt(g.M, g.N) == 4)
        launch_tiles<4>(gemm_scalar<MfmaF64, 4>, g, stream);
    else
        launch_tiles<2>(gemm_scalar<MfmaF64, 2>, g, stream);
    return hipGetLastError();
}

template <>
hipError_t launch_trailing_update<float>(const GemmArgs<float>& g, int update,
                                         hipStream_t stream)
{
    const bool big = pick_wt(g.M, g.N) == 4;
    if (update == MC_UPDATE_BF16X3) {
        if (big)
            launch_tiles<4>(gemm_bf16x3<4>, g, stream);
        else
            launch_tiles<2>(gemm_bf16x3<2>, g, stream);
    } else {
        if (big)
            launch_tiles<4>(gemm_scalar<MfmaF32, 4>, g, stream);
        else
            launch_tiles<2>(gemm_scalar<MfmaF32, 2>, g, stream);
    }
    return hipGetLastError();
}

} // namespace mc
