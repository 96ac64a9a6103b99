// mc_backward.hip -- d log|det A| / dA = A^{-T} from the stored factors.
//
// The factor call leaves A[:, perm] = L U in place: L lower triangular with
// the pivots on its diagonal (the stashed multipliers of Figure 6 step 4.8
// below it), U unit upper triangular (the factored pivot rows, steps
// 4.3-4.4).  Then A^{-1} = Q U^{-1} L^{-1} with Q the column permutation,
// and the gradient of log|det A| is A^{-T}:
//   Z = L^{-1}                   blocked forward substitution on L Z = I
//   Z <- U^{-1} Z                blocked backward substitution
//   G[j][perm[s]] = g Z[s][j]    (A^{-1} = Q Z, transposed)
// The off-diagonal block updates are the MFMA trailing-update kernel
// (mc_gemm.hip); the diagonal blocks are solved column by column with the
// block held in LDS and the column in registers.
#include <algorithm>

#include "mc_device.h"
#include "mc_gemm.h"
#include "mc_internal.h"

namespace mc {

constexpr int kBwdThreads = 256;
constexpr int kBwdBlock = 64; // block size of the substitutions

template <typename T>
__global__ void __launch_bounds__(kBwdThreads)
bwd_init(T* Z, int64_t ldz, int64_t n, int* ident, DevState* st)
{
    const int64_t i = blockIdx.x;
    for (int64_t j = threadIdx.x; j < n; j += kBwdThreads)
        Z[i * ldz + j] = (i == j) ? T(1) : T(0);
    if (i == 0) {
        for (int64_t j = threadIdx.x; j < n; j += kBwdThreads) ident[j] = (int)j;
        if (threadIdx.x == 0) {
            st->status = kStatusOk;
            st->bad_step = 0;
        }
    }
}

// Z[I0:I0+nb, 0:ncols] <- L_II^{-1} Z[...]  (L_II lower, pivots on diagonal)
template <typename T, int NB>
__global__ void __launch_bounds__(kBwdThreads)
bwd_lsolve_diag(const T* __restrict__ LU, int64_t ld, T* Z, int64_t ldz,
                int64_t I0, int nb, int64_t ncols)
{
    __shared__ T Ld[NB][NB + 1];
    for (int e = threadIdx.x; e < NB * NB; e += kBwdThreads) {
        const int r = e / NB, k = e - r * NB;
        Ld[r][k] = (r < nb && k < nb && k <= r) ? LU[(I0 + r) * ld + I0 + k] : T(0);
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * kBwdThreads + threadIdx.x;
    if (j >= ncols) return;
    T z[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) z[r] = (r < nb) ? Z[(I0 + r) * ldz + j] : T(0);
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        if (r >= nb) break;
        T acc = z[r];
#pragma unroll
        for (int k = 0; k < r; ++k) acc = fma(-Ld[r][k], z[k], acc);
        z[r] = acc / Ld[r][r];
    }
#pragma unroll
    for (int r = 0; r < NB; ++r)
        if (r < nb) Z[(I0 + r) * ldz + j] = z[r];
}

// Z[I0:I0+nb, :] <- U_II^{-1} Z[...]  (U_II unit upper)
template <typename T, int NB>
__global__ void __launch_bounds__(kBwdThreads)
bwd_usolve_diag(const T* __restrict__ LU, int64_t ld, T* Z, int64_t ldz,
                int64_t I0, int nb, int64_t ncols)
{
    __shared__ T Ud[NB][NB + 1];
    for (int e = threadIdx.x; e < NB * NB; e += kBwdThreads) {
        const int r = e / NB, k = e - r * NB;
        Ud[r][k] = (r < nb && k < nb && k > r) ? LU[(I0 + r) * ld + I0 + k] : T(0);
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * kBwdThreads + threadIdx.x;
    if (j >= ncols) return;
    T z[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) z[r] = (r < nb) ? Z[(I0 + r) * ldz + j] : T(0);
#pragma unroll
    for (int r = NB - 1; r >= 0; --r) {
        if (r >= nb) continue;
        T acc = z[r];
#pragma unroll
        for (int k = r + 1; k < NB; ++k) acc = fma(-Ud[r][k], z[k], acc);
        z[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r)
        if (r < nb) Z[(I0 + r) * ldz + j] = z[r];
}

// G[j][perm[s]] = g * Z[s][j], 32 x 32 tiles through LDS.  When the
// forward result `fwd` (optional) reports a failed factorisation (info != 0:
// singular, non-finite or aborted) the factors are not a valid L U, and every
// entry of G is NaN instead.
template <typename T>
__global__ void __launch_bounds__(kBwdThreads)
bwd_output(const T* __restrict__ Z, int64_t ldz, const int* __restrict__ perm,
           int64_t n, const double* grad_out, const mc_result* fwd, T* G,
           int64_t ldg)
{
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5; // 32 x 8
    const int64_t s0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
    T g = grad_out ? (T)(*grad_out) : T(1);
    if (fwd && fwd->info != 0) g = (T)NAN;
    for (int y = ty; y < 32; y += 8) {
        const int64_t s = s0 + y, j = j0 + tx;
        tile[y][tx] = (s < n && j < n) ? Z[s * ldz + j] : T(0);
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int64_t j = j0 + y, s = s0 + tx;
        if (j < n && s < n) {
            // perm is read only from a valid factorisation
            const int64_t c = (fwd && fwd->info != 0) ? s : perm[s];
            G[j * ldg + c] = g * tile[tx][y];
        }
    }
}

template <typename T>
static void launch_diag(bool lower, const T* LU, int64_t ld, T* Z, int64_t ldz,
                        int64_t I0, int nb, int64_t ncols, hipStream_t st)
{
    const dim3 grid((unsigned)((ncols + kBwdThreads - 1) / kBwdThreads));
    if (lower) {
        if (nb <= 16)
            hipLaunchKernelGGL((bwd_lsolve_diag<T, 16>), grid, dim3(kBwdThreads), 0, st, LU, ld, Z, ldz, I0, nb, ncols);
        else if (nb <= 32)
            hipLaunchKernelGGL((bwd_lsolve_diag<T, 32>), grid, dim3(kBwdThreads), 0, st, LU, ld, Z, ldz, I0, nb, ncols);
        else
            hipLaunchKernelGGL((bwd_lsolve_diag<T, 64>), grid, dim3(kBwdThreads), 0, st, LU, ld, Z, ldz, I0, nb, ncols);
    } else {
        if (nb <= 16)
            hipLaunchKernelGGL((bwd_usolve_diag<T, 16>), grid, dim3(kBwdThreads), 0, st, LU, ld, Z, ldz, I0, nb, ncols);
        else if (nb <= 32)
            hipLaunchKernelGGL((bwd_usolve_diag<T, 32>), grid, dim3(kBwdThreads), 0, st, LU, ld, Z, ldz, I0, nb, ncols);
        else
            hipLaunchKernelGGL((bwd_usolve_diag<T, 64>), grid, dim3(kBwdThreads), 0, st, LU, ld, Z, ldz, I0, nb, ncols);
    }
}

template <typename T>
hipError_t launch_backward(const T* LU, int64_t ld, const int* perm, int64_t n,
                           const double* grad_out, const mc_result* fwd, T* G,
                           int64_t ldg, BwdWork<T> w, hipStream_t st)
{
    const int update = MC_UPDATE_NATIVE;
    hipLaunchKernelGGL(bwd_init<T>, dim3((unsigned)n), dim3(kBwdThreads), 0, st,
                       w.Z, w.ldz, n, w.ident, w.state);
    // forward substitution L Z = I; Z = L^{-1} is lower triangular, so
    // block row I only has columns 0 .. I1-1
    for (int64_t I0 = 0; I0 < n; I0 += kBwdBlock) {
        const int nb = (int)std::min<int64_t>(kBwdBlock, n - I0);
        const int64_t I1 = I0 + nb;
        launch_diag<T>(true, LU, ld, w.Z, w.ldz, I0, nb, I1, st);
        if (I1 < n) {
            GemmArgs<T> g;
            g.C = w.Z; g.ldc = w.ldz; g.r0 = I1; g.c0 = 0;
            g.M = n - I1; g.N = I1; g.K = nb;
            g.L = LU + I1 * ld + I0; g.ldl = ld;
            g.U = w.Z + I0 * w.ldz; g.ldu = w.ldz;
            g.colsrc = w.ident; g.state = w.state;
            const hipError_t e = launch_trailing_update(g, update, st);
            if (e != hipSuccess) return e;
        }
    }
    // backward substitution U Z <- Z, bottom block row first
    const int64_t last = ((n - 1) / kBwdBlock) * kBwdBlock;
    for (int64_t I0 = last; I0 >= 0; I0 -= kBwdBlock) {
        const int nb = (int)std::min<int64_t>(kBwdBlock, n - I0);
        launch_diag<T>(false, LU, ld, w.Z, w.ldz, I0, nb, n, st);
        if (I0 > 0) {
            GemmArgs<T> g;
            g.C = w.Z; g.ldc = w.ldz; g.r0 = 0; g.c0 = 0;
            g.M = I0; g.N = n; g.K = nb;
            g.L = LU + I0; g.ldl = ld;
            g.U = w.Z + I0 * w.ldz; g.ldu = w.ldz;
            g.colsrc = w.ident; g.state = w.state;
            const hipError_t e = launch_trailing_update(g, update, st);
            if (e != hipSuccess) return e;
        }
    }
    const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
    hipLaunchKernelGGL(bwd_output<T>, grid, dim3(kBwdThreads), 0, st, w.Z, w.ldz,
                       perm, n, grad_out, fwd, G, ldg);
    return hipGetLastError();
}

template hipError_t launch_backward<double>(const double*, int64_t, const int*,
                                            int64_t, const double*,
                                            const mc_result*, double*, int64_t,
                                            BwdWork<double>, hipStream_t);
template hipError_t launch_backward<float>(const float*, int64_t, const int*,
                                           int64_t, const double*,
                                           const mc_result*, float*, int64_t,
                                           BwdWork<float>, hipStream_t);

} // namespace mc
