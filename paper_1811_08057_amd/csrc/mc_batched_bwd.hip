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
#include "mc_solve.h"

namespace mc {

namespace {

constexpr int64_t kQSortMax = 16384;

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

// One item: column block J of matrix k.
template <typename T>
__device__ void bbwd_item(const BatchedBwdArgs& a, int k, int J, T* lds)
{
    const int tid = threadIdx.x;
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

    const T* inv = reinterpret_cast<const T*>(static_cast<const unsigned char*>(a.inv) +
                                              (size_t)k * a.inv_stride);
    // Y = U^{-1} L^{-1} E_J; L^{-1} E_J is zero above block J
    lu_solve_rhs<T>(LU, ld, n, inv, Yt, ldg, w, J, true, X, As, Bs, D);
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

// The diagonal blocks' inverses of every member: block (2 B + half, k).
template <typename T>
__global__ void __launch_bounds__(kQB)
bbwd_invert(BatchedBwdArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int64_t per = 2 * qblocks(std::max<int64_t>(a.n_max, 1));
    const int k = (int)(blockIdx.x / per);
    const int64_t half = blockIdx.x - (int64_t)k * per;
    const int64_t B = half >> 1;
    const int64_t n = a.n_array[k];
    if (n < 0 || n > a.n_max || B >= qblocks(n)) return;
    if (a.fwd != nullptr && a.fwd[k].info != 0) return; // no valid factors
    T* inv = reinterpret_cast<T*>(static_cast<unsigned char*>(a.inv) + (size_t)k * a.inv_stride);
    invert_diag_block<T>(static_cast<const T*>(a.LU_array[k]), a.ld_array[k], n, B,
                         (half & 1) != 0, inv, lds, lds + kQW * kQXLD);
}

template <typename T>
__global__ void __launch_bounds__(kQB, 2)
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

static size_t inv_stride_bytes(int64_t n_max, size_t elem)
{
    return align_up(elem * 2 * kQW * kQW * (size_t)qblocks(std::max<int64_t>(n_max, 1)), 256);
}

size_t batched_bwd_workspace_bytes(int64_t batch, int64_t n_max, int dtype)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t items = std::max<int64_t>(batch, 1) * qblocks(std::max<int64_t>(n_max, 1));
    return align_up(sizeof(int) * 64, 256) +
           align_up(sizeof(int) * (size_t)std::max<int64_t>(batch, 1), 256) +
           align_up(sizeof(int) * 2 * (size_t)items, 256) +
           (size_t)std::max<int64_t>(batch, 1) * inv_stride_bytes(n_max, elem);
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
    const int64_t items_max = std::max<int64_t>(a.batch, 1) * qblocks(std::max<int64_t>(a.n_max, 1));
    p += align_up(sizeof(int) * 2 * (size_t)items_max, 256);
    a.inv = p;
    a.inv_stride = inv_stride_bytes(a.n_max, dtype == MC_DTYPE_F64 ? 8 : 4);
    const size_t lds = batched_bwd_lds_bytes(dtype, a.n_max);
    a.lds_elems = lds / (dtype == MC_DTYPE_F64 ? 8 : 4);
    hipLaunchKernelGGL(bbwd_setup, dim3(1), dim3(kQB), 0, stream, a.n_array, a.batch,
                       a.n_max, a.counter, order, a.items);
    {
        const size_t inv_lds = (dtype == MC_DTYPE_F64 ? 8 : 4) * (size_t)(2 * kQW * kQXLD);
        const void* fi = dtype == MC_DTYPE_F64 ? reinterpret_cast<const void*>(&bbwd_invert<double>)
                                               : reinterpret_cast<const void*>(&bbwd_invert<float>);
        if (inv_lds > 64 * 1024) {
            const hipError_t ea = hipFuncSetAttribute(fi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      (int)inv_lds);
            if (ea != hipSuccess) return note_hip_error(ea);
        }
        const dim3 ig((unsigned)(2 * qblocks(std::max<int64_t>(a.n_max, 1)) * a.batch));
        if (dtype == MC_DTYPE_F64)
            hipLaunchKernelGGL(bbwd_invert<double>, ig, dim3(kQB), inv_lds, stream, a);
        else
            hipLaunchKernelGGL(bbwd_invert<float>, ig, dim3(kQB), inv_lds, stream, a);
    }
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
