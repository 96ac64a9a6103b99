// mc_batched_bwd.hip -- gradients of many log-determinants in one
// persistent launch: G_k = g_k A_k^{-T} from the factors the factor calls
// keep (A_k[:, perm_k] = L_k U_k, L lower with the pivots on its diagonal,
// U unit upper; Figure 6 steps 4.3-4.4 and 4.8).
//
// A^{-1} = Q U^{-1} L^{-1}, so column block J of A^{-1}, permuted, is
//   Y = U^{-1} (L^{-1} E_J)          E_J = columns c0 .. c0+63 of I
// and G[c0 + j][perm[s]] = g Y[s][j].  One work item is one (matrix, block J)
// pair; items are independent, so the workgroups of one launch take them
// from a queue ordered largest matrix first and never wait for each other.
// An item runs two blocked substitutions by 64-row blocks: each block is a
// GEMM update on the matrix cores (K in chunks of 32 staged through LDS)
// followed by a 64 x 64 triangular solve in LDS, one lane per column.  The
// forward substitution starts at block c0 (L^{-1} E_J is zero above it).
// Y lives in the item's own rows of G (row c0 + j holds Y[.][j] in position
// order), which the last stage permutes in place: no workspace beyond the
// queue.
#include <algorithm>

#include "mc_batched_bwd.h"
#include "mc_device.h"
#include "mc_mfma.h"

namespace mc {

namespace {

constexpr int kQB = 256;       // threads per workgroup (4 wavefronts)
constexpr int kQW = 64;        // right-hand sides per item, rows per block
constexpr int kQKC = 32;       // K chunk of the block updates
constexpr int kQLD = kQKC + 1; // LDS row stride of the staged chunks
constexpr int kQXLD = kQW + 1; // LDS row stride of the 64 x 64 blocks
constexpr int64_t kQSortMax = 16384;

__host__ __device__ inline int64_t qblocks(int64_t n) { return (n + kQW - 1) / kQW; }

// One block: the matrices by decreasing size (ties by index), then their
// items (k, J) in that order; counter[0] = 0 (queue head), counter[1] =
// the number of items.
__global__ void __launch_bounds__(kQB)
bbwd_setup(const int64_t* __restrict__ n_array, int64_t batch, int64_t n_max,
           int* counter, int* order, int* items)
{
    __shared__ int64_t part[kQB];
    const int tid = threadIdx.x;
    auto nblk = [&](int64_t k) -> int64_t {
        const int64_t n = n_array[k];
        return (n < 0 || n > n_max) ? 0 : qblocks(n);
    };
    if (batch > kQSortMax) {
        for (int64_t i = tid; i < batch; i += kQB) order[i] = (int)i;
    } else {
        for (int64_t i = tid; i < batch; i += kQB) {
            const int64_t ni = n_array[i];
            int64_t rank = 0;
            for (int64_t j = 0; j < batch; ++j) {
                const int64_t nj = n_array[j];
                rank += (nj > ni || (nj == ni && j < i)) ? 1 : 0;
            }
            order[rank] = (int)i;
        }
    }
    __syncthreads();
    // contiguous chunk of the order per thread, then an exclusive scan
    const int64_t per = (batch + kQB - 1) / kQB;
    const int64_t lo = std::min<int64_t>(batch, tid * per);
    const int64_t hi = std::min<int64_t>(batch, lo + per);
    int64_t sum = 0;
    for (int64_t q = lo; q < hi; ++q) sum += nblk(order[q]);
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        int64_t run = 0;
        for (int t = 0; t < kQB; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        counter[0] = 0;
        counter[1] = (int)run;
    }
    __syncthreads();
    int64_t at = part[tid];
    for (int64_t q = lo; q < hi; ++q) {
        const int k = order[q];
        const int64_t nb = nblk(k);
        for (int64_t J = 0; J < nb; ++J, ++at) {
            items[2 * at] = k;
            items[2 * at + 1] = (int)J;
        }
    }
}

struct QShared {
    int q;
};

// acc (this wave's 16 rows x 64 columns of the block) -= A[rows, K] B[K, cols]
// over K in [k_lo, k_hi): A from `a_rows` (row-major, stride lda, rows
// r0 .. r0+63 valid below r_end), B from the transposed store Yt (row j =
// column j of B, stride ldy, columns j < w valid).
template <typename T>
__device__ void block_update(const T* __restrict__ Amat, int64_t lda, int64_t r0,
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
__device__ void lower_solve(const T* D, T* X, int lane)
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
__device__ void unit_upper_solve(const T* D, T* X, int lane)
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

// One item: column block J of matrix k.
template <typename T>
__device__ void bbwd_item(const BatchedBwdArgs& a, int k, int J, T* lds)
{
    using P = typename MfmaFor<T>::P;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = a.n_array[k];
    const int64_t c0 = (int64_t)J * kQW;
    const int w = (int)std::min<int64_t>(kQW, n - c0);
    T* G = static_cast<T*>(a.G_array[k]);
    const int64_t ldg = a.ldg_array[k];
    T* Yt = G + c0 * ldg; // row j: Y[.][j] in position order
    const bool failed = a.fwd != nullptr && a.fwd[k].info != 0;
    if (failed) { // the factors are not a valid L U
        for (int j = 0; j < w; ++j)
            for (int64_t s = tid; s < n; s += kQB) Yt[j * ldg + s] = (T)NAN;
        return;
    }
    const T* LU = static_cast<const T*>(a.LU_array[k]);
    const int64_t ld = a.ld_array[k];
    const T g = a.grad_out ? (T)a.grad_out[k] : T(1);
    T* X = lds;                    // [64][kQXLD] the block being solved
    T* As = X + kQW * kQXLD;       // [64][kQLD]
    T* Bs = As + kQW * kQLD;       // [64][kQLD]
    T* D = As;                     // [64][kQXLD] diagonal block (aliases As, Bs)
    const int ci = lane & 15;

    auto to_x = [&](typename P::Acc (&acc)[4], int64_t I0, bool from_y, bool ident) {
        // X = (identity / Y block) - acc; rows past n and columns past w are 0
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * wv + P::drow(lane, q), j = 16 * t + ci;
                const int64_t row = I0 + r;
                T v = T(0);
                if (row < n && j < w) {
                    if (ident) v = (row == c0 + j) ? T(1) : T(0);
                    if (from_y) v = Yt[(int64_t)j * ldg + row];
                    v -= acc[t][q];
                }
                X[r * kQXLD + j] = v;
            }
    };
    auto store_x = [&](int64_t I0) {
        for (int e = tid; e < kQW * kQW; e += kQB) {
            const int j = e >> 6, r = e & 63;
            if (j < w && I0 + r < n) Yt[(int64_t)j * ldg + I0 + r] = X[r * kQXLD + j];
        }
    };
    const int64_t nblk = qblocks(n);

    // forward substitution L Y = E_J, from block J on
    for (int64_t B = J; B < nblk; ++B) {
        const int64_t I0 = B * kQW;
        typename P::Acc acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = typename P::Acc{0, 0, 0, 0};
        block_update<T>(LU, ld, I0, n, Yt, ldg, w, c0, I0, As, Bs, acc);
        to_x(acc, I0, false, true);
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
    // backward substitution U Y <- Y, last block first (rows above c0 start
    // from zero)
    for (int64_t B = nblk - 1; B >= 0; --B) {
        const int64_t I0 = B * kQW;
        typename P::Acc acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = typename P::Acc{0, 0, 0, 0};
        block_update<T>(LU, ld, I0, n, Yt, ldg, w, I0 + kQW, n, As, Bs, acc);
        to_x(acc, I0, B >= J, false);
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
    // G[c0 + j][perm[s]] = g Y[s][j]: each row through LDS, then scattered
    const int32_t* perm = a.perm_array[k];
    T* buf = lds;
    const int64_t cap = (int64_t)(a.lds_elems);
    const int rows_at_once = (int)std::max<int64_t>(1, std::min<int64_t>(w, cap / std::max<int64_t>(n, 1)));
    for (int j0 = 0; j0 < w; j0 += rows_at_once) {
        const int jr = std::min(rows_at_once, w - j0);
        for (int64_t e = tid; e < (int64_t)jr * n; e += kQB) {
            const int jj = (int)(e / n);
            const int64_t s = e - (int64_t)jj * n;
            buf[e] = Yt[(int64_t)(j0 + jj) * ldg + s];
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)jr * n; e += kQB) {
            const int jj = (int)(e / n);
            const int64_t s = e - (int64_t)jj * n;
            Yt[(int64_t)(j0 + jj) * ldg + perm[s]] = g * buf[e];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kQB)
bbwd_persistent(BatchedBwdArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ QShared sh;
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int total = a.counter[1];
    for (;;) {
        if (threadIdx.x == 0) sh.q = atomicAdd(a.counter, 1);
        __syncthreads();
        const int q = sh.q;
        __syncthreads();
        if (q >= total) break;
        bbwd_item<T>(a, a.items[2 * q], a.items[2 * q + 1], lds);
        __syncthreads();
    }
}

} // namespace

size_t batched_bwd_lds_bytes(int dtype, int64_t n_max)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const size_t solve = elem * (size_t)(kQW * kQXLD + 2 * kQW * kQLD);
    const size_t row = elem * (size_t)std::max<int64_t>(n_max, 1);
    return std::max(solve, row);
}

size_t batched_bwd_workspace_bytes(int64_t batch, int64_t n_max)
{
    const int64_t items = std::max<int64_t>(batch, 1) * qblocks(std::max<int64_t>(n_max, 1));
    return align_up(sizeof(int) * 64, 256) +
           align_up(sizeof(int) * (size_t)std::max<int64_t>(batch, 1), 256) +
           align_up(sizeof(int) * 2 * (size_t)items, 256);
}

hipError_t launch_batched_backward(BatchedBwdArgs a, int dtype, void* work,
                                   hipStream_t stream)
{
    unsigned char* p = static_cast<unsigned char*>(work);
    a.counter = reinterpret_cast<int*>(p);
    p += align_up(sizeof(int) * 64, 256);
    int* order = reinterpret_cast<int*>(p);
    p += align_up(sizeof(int) * (size_t)std::max<int64_t>(a.batch, 1), 256);
    a.items = reinterpret_cast<int*>(p);
    const size_t lds = batched_bwd_lds_bytes(dtype, a.n_max);
    a.lds_elems = lds / (dtype == MC_DTYPE_F64 ? 8 : 4);
    hipLaunchKernelGGL(bbwd_setup, dim3(1), dim3(kQB), 0, stream, a.n_array, a.batch,
                       a.n_max, a.counter, order, a.items);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return note_hip_error(e);
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return note_hip_error(e);
    const int64_t most = a.batch * qblocks(std::max<int64_t>(a.n_max, 1));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2 * (int64_t)cus, most));
    const void* f = dtype == MC_DTYPE_F64 ? reinterpret_cast<const void*>(&bbwd_persistent<double>)
                                          : reinterpret_cast<const void*>(&bbwd_persistent<float>);
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return note_hip_error(e);
    }
    if (dtype == MC_DTYPE_F64)
        hipLaunchKernelGGL(bbwd_persistent<double>, dim3(grid), dim3(kQB), lds, stream, a);
    else
        hipLaunchKernelGGL(bbwd_persistent<float>, dim3(grid), dim3(kQB), lds, stream, a);
    return note_hip_error(hipGetLastError());
}

} // namespace mc
