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

#include "mc_mfma.h"

namespace mc {

constexpr int kQB = 256;       // threads per workgroup (4 wavefronts)
constexpr int kQW = 64;        // right-hand sides per item, rows per block
constexpr int kQKC = 32;       // K chunk of the block updates
constexpr int kQLD = kQKC + 1; // LDS row stride of the staged chunks
constexpr int kQXLD = kQW + 1; // LDS row stride of the 64 x 64 blocks

__host__ __device__ inline int64_t qblocks(int64_t n) { return (n + kQW - 1) / kQW; }

// acc (this wave's 16 rows x 64 columns of the block) -= A[rows, K] B[K, cols]
// over K in [k_lo, k_hi): A from `a_rows` (row-major, stride lda, rows
// r0 .. r0+63 valid below r_end), B from the transposed store Yt (row j =
// column j of B, stride ldy, columns j < w valid).
template <typename T>
__device__ inline void block_update(const T* __restrict__ Amat, int64_t lda, int64_t r0,
                             int64_t r_end, const T* Yt, int64_t ldy, int w,
                             int64_t k_lo, int64_t k_hi, T* As, T* Bs,
                             typename MfmaFor<T>::P::Acc (&acc)[4])
{
    using P = typename MfmaFor<T>::P;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ci = lane & 15, kq = lane >> 4;
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += kQKC) {
#pragma unroll
        for (int u = 0; u < kQW * kQKC / kQB; ++u) {
            const int e = tid + kQB * u;
            const int r = e / kQKC, kk = e - r * kQKC;
            const int64_t k = k0 + kk;
            const bool kin = k < k_hi;
            const int64_t row = r0 + r;
            As[r * kQLD + kk] = (kin && row < r_end) ? Amat[row * lda + k] : T(0);
            Bs[r * kQLD + kk] = (kin && r < w) ? Yt[(int64_t)r * ldy + k] : T(0);
        }
        __syncthreads();
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
// diagonal (the pivots); lane j solves column j.  By 16-row sub-blocks: the
// sub-block's rows in registers, then its contribution to the rows below.
template <typename T>
__device__ inline void lower_solve(const T* D, T* X, int lane)
{
    for (int sb = 0; sb < kQW / 16; ++sb) {
        T x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = 16 * sb + i;
            T s = X[r * kQXLD + lane];
#pragma unroll
            for (int c = 0; c < i; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], x[c], s);
            x[i] = s / D[r * kQXLD + r];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) X[(16 * sb + i) * kQXLD + lane] = x[i];
        for (int r = 16 * (sb + 1); r < kQW; ++r) {
            T s = X[r * kQXLD + lane];
#pragma unroll
            for (int c = 0; c < 16; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], x[c], s);
            X[r * kQXLD + lane] = s;
        }
    }
}

// X <- D^{-1} X with D unit upper triangular (its strict upper part given).
template <typename T>
__device__ inline void unit_upper_solve(const T* D, T* X, int lane)
{
    for (int sb = kQW / 16 - 1; sb >= 0; --sb) {
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
        for (int r = 0; r < 16 * sb; ++r) {
            T s = X[r * kQXLD + lane];
#pragma unroll
            for (int c = 0; c < 16; ++c) s = fma(-D[r * kQXLD + 16 * sb + c], x[c], s);
            X[r * kQXLD + lane] = s;
        }
    }
}

// Y <- U^{-1} L^{-1} Y for the w <= 64 right-hand sides in Yt (row j holds
// right-hand side j over positions 0..n-1, stride ldy), with the factors
// LU (row stride ld).  first = J and ident: the right-hand sides are
// columns 64 J .. 64 J + w - 1 of the identity (Yt's contents are not read;
// L^{-1} E_J is zero above block J, so the forward substitution starts
// there).  first = 0 and !ident: Yt holds the right-hand sides.  X, As, Bs,
// D: LDS (64 x kQXLD, 64 x kQLD twice, 64 x kQXLD; D may alias As and Bs).
// Called by the whole workgroup; ends with a barrier.
template <typename T>
__device__ inline void lu_solve_rhs(const T* __restrict__ LU, int64_t ld, int64_t n,
                                    T* Yt, int64_t ldy, int w, int64_t first,
                                    bool ident, T* X, T* As, T* Bs, T* D)
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
        for (int e = tid; e < kQW * kQW; e += kQB) { // L_II, identity past n
            const int r = e >> 6, c = e & 63;
            const int64_t row = I0 + r;
            T v = T(0);
            if (row < n) {
                if (c <= r) v = LU[row * ld + I0 + c];
            } else if (c == r) {
                v = T(1);
            }
            D[r * kQXLD + c] = v;
        }
        __syncthreads();
        if (wv == 0) lower_solve(D, X, lane);
        __syncthreads();
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
        for (int e = tid; e < kQW * kQW; e += kQB) { // strict upper part of U_II
            const int r = e >> 6, c = e & 63;
            const int64_t row = I0 + r;
            D[r * kQXLD + c] = (row < n && c > r && I0 + c < n) ? LU[row * ld + I0 + c] : T(0);
        }
        __syncthreads();
        if (wv == 0) unit_upper_solve(D, X, lane);
        __syncthreads();
        store_x(I0);
        __syncthreads();
    }
}

} // namespace mc
