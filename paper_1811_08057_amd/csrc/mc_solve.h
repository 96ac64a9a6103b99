// mc_solve.h -- device pieces of the blocked triangular substitutions with
// many right-hand sides, shared by the batched backward (columns of A^{-1})
// and the mixture log-likelihood (Mahalanobis terms) on the factors the
// factor calls keep: A[:, perm] = L U, L lower with the pivots on its
// diagonal, U unit upper (Figure 6 steps 4.3-4.4 and 4.8).
//
// A work item solves for 64 right-hand sides held transposed (row j of Yt
// is right-hand side j, in position order) by 64-row blocks: a block update
// on the matrix cores (K in chunks of 32 staged through LDS), then the
// 64 x 64 triangular solve of the block in LDS, one lane per right-hand side.
#pragma once

#include <hip/hip_runtime.h>

#include "mc_device.h"
#include "mc_mfma.h"

namespace mc {

constexpr int kQB = 256;       // threads per workgroup (4 wavefronts)
constexpr int kQW = 64;        // right-hand sides per item, rows per block
constexpr int kQKC = 32;       // K chunk of the block updates
constexpr int kQLD = kQKC + 1; // LDS row stride of the staged chunks
constexpr int kQXLD = kQW + 1; // LDS row stride of the 64 x 64 blocks

__host__ __device__ inline int64_t qblocks(int64_t n) { return (n + kQW - 1) / kQW; }

// acc (this wave's 16 rows x 64 columns of the block) -= A[rows, K] B[K, cols]
// over K in [k_lo, k_hi): A from Amat (row-major, stride lda, rows r0 ..
// r0+63, valid below r_end), B from the transposed store Yt (row j = column
// j of B, stride ldy, columns j < w valid).  The next chunk is read into
// registers while the matrix cores work on this one; one LDS buffer, two
// barriers per chunk.
template <typename T>
__device__ inline void block_update(const T* __restrict__ Amat, int64_t lda, int64_t r0,
                                    int64_t r_end, const T* Yt, int64_t ldy, int w,
                                    int64_t k_lo, int64_t k_hi, T* As, T* Bs,
                                    typename MfmaFor<T>::P::Acc (&acc)[4])
{
    using P = typename MfmaFor<T>::P;
    constexpr int PER = kQW * kQKC / kQB; // elements of each operand a thread moves
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ci = lane & 15, kq = lane >> 4;
    if (k_lo >= k_hi) return;
    T pa[PER], pb[PER];
    // the block's 64 rows of A from column 0 and the w rows of Yt, through
    // buffer descriptors (an element past a row's K range or past the rows
    // reads 0: no branch, and the loads go out together)
    const int64_t arows = (r_end - r0) < kQW ? (r_end - r0) : kQW;
    const __amdgpu_buffer_rsrc_t ra =
        operand_rsrc(Amat + r0 * lda, sizeof(T) * ((arows - 1) * lda + k_hi));
    const __amdgpu_buffer_rsrc_t rb = operand_rsrc(Yt, sizeof(T) * ((int64_t)(w - 1) * ldy + k_hi));
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + kQB * u;
            const int r = e / kQKC, kk = e - r * kQKC;
            const int64_t k = k0 + kk;
            const bool kin = k < k_hi;
            pa[u] = operand_load<T>(
                ra, (kin && r < arows) ? (uint32_t)(sizeof(T) * (r * lda + k)) : kOutOfRange);
            pb[u] = operand_load<T>(
                rb, (kin && r < w) ? (uint32_t)(sizeof(T) * ((int64_t)r * ldy + k)) : kOutOfRange);
        }
    };
    gload(k_lo);
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += kQKC) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + kQB * u;
            const int r = e / kQKC, kk = e - r * kQKC;
            As[r * kQLD + kk] = pa[u];
            Bs[r * kQLD + kk] = pb[u];
        }
        __syncthreads();
        if (k0 + kQKC < k_hi) gload(k0 + kQKC);
#pragma unroll
        for (int kk = 0; kk < kQKC; kk += 4) {
            const T a = As[(16 * wv + ci) * kQLD + kk + kq];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const T b = Bs[(16 * t + ci) * kQLD + kk + kq];
                acc[t] = P::mma(a, b, acc[t]);
            }
        }
        __syncthreads();
    }
}

// X <- D^{-1} X for the 64 x 64 block in LDS, D lower triangular with its
// diagonal (the pivots), by 16-row sub-blocks: wavefront 0 solves the
// sub-block's rows (lane j for right-hand side j, multiplying by the
// pivots' reciprocals in rinv), then all four wavefronts apply the
// sub-block to the rows below it, a row each in turn.  Called by the whole
// workgroup (barriers inside).
template <typename T>
__device__ inline void lower_solve(const T* D, const T* rinv, T* X)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int sb = 0; sb < kQW / 16; ++sb) {
        if (wv == 0) {
            T x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = 16 * sb + i;
                T s = X[r * kQXLD + lane];
#pragma unroll
                for (int c = 0; c < i; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], x[c], s);
                x[i] = s * rinv[r];
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) X[(16 * sb + i) * kQXLD + lane] = x[i];
        }
        __syncthreads();
        T xs[16]; // the sub-block's solution, read once
#pragma unroll
        for (int c = 0; c < 16; ++c) xs[c] = X[(16 * sb + c) * kQXLD + lane];
        for (int r = 16 * (sb + 1) + wv; r < kQW; r += kQB / 64) {
            T s = X[r * kQXLD + lane];
#pragma unroll
            for (int c = 0; c < 16; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], xs[c], s);
            X[r * kQXLD + lane] = s;
        }
        __syncthreads();
    }
}

// X <- D^{-1} X with D unit upper triangular (its strict upper part given),
// last sub-block first; otherwise as lower_solve.
template <typename T>
__device__ inline void unit_upper_solve(const T* D, T* X)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int sb = kQW / 16 - 1; sb >= 0; --sb) {
        if (wv == 0) {
            T x[16];
#pragma unroll
            for (int i = 15; i >= 0; --i) {
                const int r = 16 * sb + i;
                T s = X[r * kQXLD + lane];
#pragma unroll
                for (int c = i + 1; c < 16; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], x[c], s);
                x[i] = s;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) X[(16 * sb + i) * kQXLD + lane] = x[i];
        }
        __syncthreads();
        T xs[16]; // the sub-block's solution, read once
#pragma unroll
        for (int c = 0; c < 16; ++c) xs[c] = X[(16 * sb + c) * kQXLD + lane];
        for (int r = wv; r < 16 * sb; r += kQB / 64) {
            T s = X[r * kQXLD + lane];
#pragma unroll
            for (int c = 0; c < 16; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], xs[c], s);
            X[r * kQXLD + lane] = s;
        }
        __syncthreads();
    }
}

// The inverses of the 64 x 64 diagonal blocks of one matrix's factors,
// shared by every work item of that matrix: block B's lower inverse
// (L_BB^{-1}, the pivots on L's diagonal) at inv + 2 B kQW^2, its unit upper
// inverse (U_BB^{-1}) at inv + (2 B + 1) kQW^2, row-major 64 x 64; rows
// and columns past n hold the identity.  One workgroup per (block, half):
// the block's triangular solve with the identity as right-hand sides.
template <typename T>
__device__ inline void invert_diag_block(const T* __restrict__ LU, int64_t ld, int64_t n,
                                         int64_t B, bool upper, T* inv, T* X, T* D)
{
    __shared__ T rinv2[kQW];
    const int tid = threadIdx.x;
    const int64_t I0 = B * kQW;
    for (int e = tid; e < kQW * kQW; e += kQB) {
        const int r = e >> 6, c = e & 63;
        const int64_t row = I0 + r;
        T v = T(0);
        if (upper) {
            if (row < n && c > r && I0 + c < n) v = LU[row * ld + I0 + c];
        } else if (row < n) {
            if (c <= r) v = LU[row * ld + I0 + c];
        } else if (c == r) {
            v = T(1);
        }
        D[r * kQXLD + c] = v;
        X[r * kQXLD + c] = (r == c) ? T(1) : T(0);
    }
    __syncthreads();
    if (upper) {
        unit_upper_solve(D, X);
    } else {
        if (tid < kQW) rinv2[tid] = T(1) / D[tid * kQXLD + tid];
        __syncthreads();
        lower_solve(D, rinv2, X);
    }
    T* out = inv + (2 * B + (upper ? 1 : 0)) * kQW * kQW;
    for (int e = tid; e < kQW * kQW; e += kQB) out[e] = X[(e >> 6) * kQXLD + (e & 63)];
    __syncthreads();
}

// X <- Dinv X for the 64 x 64 block X in LDS, Dinv a 64 x 64 row-major
// block in global memory (a diagonal block's inverse): staged into D (LDS),
// then a 64 x 64 x 64 product on the matrix cores, four wavefronts of
// 16 rows.  Called by the whole workgroup (barriers inside).
template <typename T>
__device__ inline void block_times_inverse(const T* __restrict__ Dinv, T* D, T* X)
{
    using P = typename MfmaFor<T>::P;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ci = lane & 15, kq = lane >> 4;
    for (int e = tid; e < kQW * kQW; e += kQB) D[(e >> 6) * kQXLD + (e & 63)] = Dinv[e];
    __syncthreads();
    typename P::Acc acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = typename P::Acc{0, 0, 0, 0};
#pragma unroll 4
    for (int kk = 0; kk < kQW; kk += 4) {
        const T a = D[(16 * wv + ci) * kQXLD + kk + kq];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const T b = X[(kk + kq) * kQXLD + 16 * t + ci];
            acc[t] = P::mma(a, b, acc[t]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            X[(16 * wv + P::drow(lane, q)) * kQXLD + 16 * t + ci] = acc[t][q];
    __syncthreads();
}

// Y <- U^{-1} L^{-1} Y for the w <= 64 right-hand sides in Yt (row j holds
// right-hand side j over positions 0..n-1, stride ldy), with the factors
// LU (row stride ld) and their diagonal blocks' inverses `inv`
// (invert_diag_block).  first = J and ident: the right-hand sides are
// columns 64 J .. 64 J + w - 1 of the identity (Yt's contents are not read;
// L^{-1} E_J is zero above block J, so the forward substitution starts
// there).  first = 0 and !ident: Yt holds the right-hand sides.  X, As, Bs,
// D: LDS (64 x kQXLD, 64 x kQLD twice, 64 x kQXLD; D may alias As and Bs).
// Called by the whole workgroup; ends with a barrier.
template <typename T>
__device__ inline void lu_solve_rhs(const T* __restrict__ LU, int64_t ld, int64_t n,
                                    const T* __restrict__ inv, T* Yt, int64_t ldy, int w,
                                    int64_t first, bool ident, T* X, T* As, T* Bs, T* D)
{
    using P = typename MfmaFor<T>::P;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ci = lane & 15;
    const int64_t c0 = first * kQW;
    auto to_x = [&](typename P::Acc (&acc)[4], int64_t I0, bool from_y, bool id) {
        // X = (identity / Y block) - acc; rows past n and columns past w are 0
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * wv + P::drow(lane, q), j = 16 * t + ci;
                const int64_t row = I0 + r;
                T v = T(0);
                if (row < n && j < w) {
                    if (id) v = (row == c0 + j) ? T(1) : T(0);
                    if (from_y) v = Yt[(int64_t)j * ldy + row];
                    v -= acc[t][q];
                }
                X[r * kQXLD + j] = v;
            }
    };
    auto store_x = [&](int64_t I0) {
        for (int e = tid; e < kQW * kQW; e += kQB) {
            const int j = e >> 6, r = e & 63;
            if (j < w && I0 + r < n) Yt[(int64_t)j * ldy + I0 + r] = X[r * kQXLD + j];
        }
    };
    const int64_t nblk = qblocks(n);

    // forward substitution L Y = R, from block `first` on
    for (int64_t B = first; B < nblk; ++B) {
        const int64_t I0 = B * kQW;
        typename P::Acc acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = typename P::Acc{0, 0, 0, 0};
        block_update<T>(LU, ld, I0, n, Yt, ldy, w, c0, I0, As, Bs, acc);
        to_x(acc, I0, !ident, ident);
        block_times_inverse(inv + 2 * B * kQW * kQW, D, X); // L_BB^{-1}
        store_x(I0);
        __syncthreads();
    }
    // backward substitution U Y <- Y, last block first (with identity
    // right-hand sides, the rows above block `first` start from zero)
    for (int64_t B = nblk - 1; B >= 0; --B) {
        const int64_t I0 = B * kQW;
        typename P::Acc acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = typename P::Acc{0, 0, 0, 0};
        block_update<T>(LU, ld, I0, n, Yt, ldy, w, I0 + kQW, n, As, Bs, acc);
        to_x(acc, I0, B >= first, false);
        block_times_inverse(inv + (2 * B + 1) * kQW * kQW, D, X); // U_BB^{-1}
        store_x(I0);
        __syncthreads();
    }
}

} // namespace mc
