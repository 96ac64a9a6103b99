// mc_gmm.hip -- log-likelihood of a Gaussian mixture from the factors of its
// covariances (the use the paper gives for the log-determinant: the
// log-likelihood of model mixtures, Abstract).
//
//   l(x) = log sum_k exp( log pi_k - (d log 2 pi + log|Sigma_k| + q_k(x)) / 2 )
//   q_k(x) = (x - mu_k)^T Sigma_k^{-1} (x - mu_k)
//
// log|Sigma_k| is the factor call's result; with Sigma_k[:, perm] = L U,
// Sigma_k^{-1} = Q U^{-1} L^{-1}, so for r = x - mu_k
//   q_k(x) = sum_s r[perm[s]] (U^{-1} L^{-1} r)[s].
// One work item is one (component, block of 64 points) pair: the 64
// residuals as right-hand sides of the two blocked substitutions (block
// updates on the matrix cores), then one dot product per point with its
// permuted residual.  Items come from a queue, so the launch is one
// persistent wave of workgroups, each with its own slot of the workspace
// for the right-hand sides.  A second launch forms l(x) per point (FP64,
// shifted by the largest term) and a third sums the points.
#include <algorithm>
#include <cmath>

#include "mc_device.h"
#include "mc_gmm.h"
#include "mc_solve.h"

namespace mc {

namespace {

struct GShared {
    int q;
};

template <typename T>
__device__ void gmm_item(const GmmArgs& a, int k, int P0, T* lds, T* slot)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t d = a.d;
    const int64_t p0 = (int64_t)P0 * kQW;
    const int w = (int)std::min<int64_t>(kQW, a.m - p0);
    const mc_result* f = a.fwd + k;
    double* qout = a.Q + (int64_t)k * a.m + p0;
    if (f->info != 0 || !(f->sign > 0.0)) { // not a covariance: no value
        for (int j = tid; j < w; j += kQB) qout[j] = NAN;
        return;
    }
    const T* X = static_cast<const T*>(a.X);
    const T* mu = static_cast<const T*>(a.means) + (int64_t)k * a.ldmu;
    const T* LU = static_cast<const T*>(a.LU_array[k]);
    const int64_t ld = a.ld_array[k];
    const int32_t* perm = a.perm_array[k];
    const int64_t ldy = a.ldy;
    // right-hand side j: the residual of point p0 + j, in position order of
    // the unpermuted columns (the substitutions see positions 0..d-1); each
    // thread's eight loads of a round go out together
    for (int64_t e0 = tid; e0 < (int64_t)w * d; e0 += 8 * kQB) {
        T xv[8], mv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t e = e0 + u * kQB;
            const int j = (int)(e / d);
            const int64_t s = e - (int64_t)j * d;
            const bool in = e < (int64_t)w * d;
            xv[u] = in ? X[(p0 + j) * a.ldx + s] : T(0);
            mv[u] = in ? mu[s] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t e = e0 + u * kQB;
            const int j = (int)(e / d);
            const int64_t s = e - (int64_t)j * d;
            if (e < (int64_t)w * d) slot[j * ldy + s] = xv[u] - mv[u];
        }
    }
    __syncthreads();
    T* Xl = lds;
    T* As = Xl + kQW * kQXLD;
    T* Bs = As + kQW * kQLD;
    const T* inv = reinterpret_cast<const T*>(static_cast<const unsigned char*>(a.inv) +
                                              (size_t)k * a.inv_stride);
    lu_solve_rhs<T>(LU, ld, d, inv, slot, ldy, w, 0, false, Xl, As, Bs, As);
    // q_j = sum_s r_j[perm[s]] y_j[s]: wavefront wv takes points wv + 4 i,
    // positions in rounds of 8 a lane whose loads go out together; with
    // d <= 512 (one round) the column sources and the mean's entries there
    // are read once for all the points
    const __amdgpu_buffer_rsrc_t rperm = operand_rsrc(perm, sizeof(int32_t) * d);
    auto round_sources = [&](int64_t s0, int (&cv)[8], T (&mv)[8]) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t sidx = s0 + lane + u * kWave;
            cv[u] = (int)__builtin_amdgcn_raw_buffer_load_b32(
                rperm, sidx < d ? (uint32_t)(sizeof(int32_t) * sidx) : kOutOfRange, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) mv[u] = mu[cv[u]]; // past d: column 0, weight 0 below
    };
    auto round_sum = [&](int64_t s0, int j, const int (&cv)[8], const T (&mv)[8]) {
        const T* rx = X + (p0 + j) * a.ldx;
        const __amdgpu_buffer_rsrc_t ry = operand_rsrc(slot + j * ldy, sizeof(T) * d);
        T xv[8], yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t sidx = s0 + lane + u * kWave;
            xv[u] = rx[cv[u]];
            yv[u] = operand_load<T>(ry, sidx < d ? (uint32_t)(sizeof(T) * sidx) : kOutOfRange);
        }
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (double)(xv[u] - mv[u]) * (double)yv[u];
        return acc;
    };
    int cv0[8];
    T mv0[8];
    round_sources(0, cv0, mv0);
    for (int j = wv; j < w; j += kQB / kWave) {
        double acc = round_sum(0, j, cv0, mv0);
        for (int64_t s0 = 8 * kWave; s0 < d; s0 += 8 * kWave) {
            int cv[8];
            T mv[8];
            round_sources(s0, cv, mv);
            acc += round_sum(s0, j, cv, mv);
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) qout[j] = acc;
    }
    __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kQB, 2)
gmm_items(GmmArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ GShared sh;
    T* lds = reinterpret_cast<T*>(smem_raw);
    T* slot = static_cast<T*>(a.slots) + (size_t)blockIdx.x * kQW * a.ldy;
    const int64_t pb = qblocks(a.m);
    const int64_t total = pb * a.k;
    for (;;) {
        if (threadIdx.x == 0) sh.q = atomicAdd(a.counter, 1);
        __syncthreads();
        const int64_t q = sh.q;
        __syncthreads();
        if (q >= total) break;
        // component-major: the workgroups at work at any time share one
        // or two components, whose factors then stay in the L2
        gmm_item<T>(a, (int)(q / pb), (int)(q % pb), lds, slot);
    }
}

__global__ void gmm_reset(int* counter) { *counter = 0; }

// The diagonal blocks' inverses of every component (one workgroup per
// block and half; components that are not covariances are skipped).
template <typename T>
__global__ void __launch_bounds__(kQB)
gmm_invert(GmmArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int64_t per = 2 * qblocks(a.d);
    const int64_t k = blockIdx.x / per, half = blockIdx.x - k * per;
    const mc_result* f = a.fwd + k;
    if (f->info != 0 || !(f->sign > 0.0)) return;
    T* inv = reinterpret_cast<T*>(static_cast<unsigned char*>(a.inv) + (size_t)k * a.inv_stride);
    invert_diag_block<T>(static_cast<const T*>(a.LU_array[k]), a.ld_array[k], a.d, half >> 1,
                         (half & 1) != 0, inv, lds, lds + kQW * kQXLD);
}

// l(x_i) from the Mahalanobis terms, one thread per point; per-block sums
// for the total.
__global__ void __launch_bounds__(kQB)
gmm_points(GmmArgs a)
{
    __shared__ double part[kQB];
    const int64_t i = (int64_t)blockIdx.x * kQB + threadIdx.x;
    const double c = (double)a.d * 1.8378770664093454835606594728112; // d log(2 pi)
    double li = 0.0;
    if (i < a.m) {
        double top = -INFINITY;
        bool bad = false;
        for (int64_t k = 0; k < a.k; ++k) {
            const double q = a.Q[k * a.m + i];
            const double t = a.log_weights[k] - 0.5 * (c + a.fwd[k].logabsdet + q);
            bad = bad || !isfinite(t);
            top = fmax(top, t);
        }
        double sum = 0.0;
        for (int64_t k = 0; k < a.k; ++k) {
            const double q = a.Q[k * a.m + i];
            const double t = a.log_weights[k] - 0.5 * (c + a.fwd[k].logabsdet + q);
            sum += exp(t - top);
        }
        li = bad ? NAN : top + log(sum);
        a.loglik[i] = li;
    }
    part[threadIdx.x] = li;
    __syncthreads();
    for (int off = kQB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(kQB)
gmm_total(const double* partial, int64_t blocks, double* total)
{
    __shared__ double part[kQB];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < blocks; b += kQB) s += partial[b];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = kQB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = part[0];
}

int64_t gmm_grid(int64_t items)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        cus = 256;
    }
    return std::max<int64_t>(1, std::min<int64_t>(2 * (int64_t)cus, items));
}

} // namespace

int64_t gmm_ldy(int64_t d) { return (d + 15) / 16 * 16; }

static size_t gmm_inv_stride(int64_t d, size_t elem)
{
    return align_up(elem * 2 * kQW * kQW * (size_t)qblocks(d), 256);
}

size_t gmm_workspace_bytes(int64_t m, int64_t d, int64_t k, int dtype)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t items = qblocks(m) * k;
    const int64_t grid = 2 * 256; // at most two workgroups per compute unit
    const int64_t slots = std::min<int64_t>(grid, std::max<int64_t>(items, 1));
    const int64_t pblocks = (m + kQB - 1) / kQB;
    return align_up(sizeof(int) * 64, 256) +
           align_up(sizeof(double) * (size_t)std::max<int64_t>(m * k, 1), 256) +
           align_up(sizeof(double) * (size_t)std::max<int64_t>(pblocks, 1), 256) +
           align_up(elem * (size_t)slots * kQW * (size_t)gmm_ldy(d), 256) +
           (size_t)k * gmm_inv_stride(d, elem);
}

hipError_t launch_gmm(GmmArgs a, int dtype, void* work, size_t work_bytes,
                      hipStream_t stream)
{
    (void)work_bytes;
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    unsigned char* p = static_cast<unsigned char*>(work);
    a.counter = reinterpret_cast<int*>(p);
    p += align_up(sizeof(int) * 64, 256);
    a.Q = reinterpret_cast<double*>(p);
    p += align_up(sizeof(double) * (size_t)std::max<int64_t>(a.m * a.k, 1), 256);
    a.partial = reinterpret_cast<double*>(p);
    const int64_t pblocks = std::max<int64_t>(1, (a.m + kQB - 1) / kQB);
    p += align_up(sizeof(double) * (size_t)std::max<int64_t>(pblocks, 1), 256);
    a.slots = p;
    a.ldy = gmm_ldy(a.d);
    const int64_t nslots = std::min<int64_t>(2 * 256, std::max<int64_t>(qblocks(a.m) * a.k, 1));
    p += align_up(elem * (size_t)nslots * kQW * (size_t)a.ldy, 256);
    a.inv = p;
    a.inv_stride = gmm_inv_stride(a.d, elem);
    const int64_t items = qblocks(a.m) * a.k;
    const int64_t grid = std::min<int64_t>(gmm_grid(items), 2 * 256);
    const size_t lds = elem * (size_t)(kQW * kQXLD + 2 * kQW * kQLD);
    hipLaunchKernelGGL(gmm_reset, dim3(1), dim3(1), 0, stream, a.counter);
    {
        const size_t inv_lds = elem * (size_t)(2 * kQW * kQXLD);
        const void* fi = dtype == MC_DTYPE_F64 ? reinterpret_cast<const void*>(&gmm_invert<double>)
                                               : reinterpret_cast<const void*>(&gmm_invert<float>);
        if (inv_lds > 64 * 1024) {
            const hipError_t e = hipFuncSetAttribute(fi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)inv_lds);
            if (e != hipSuccess) return note_hip_error(e);
        }
        const dim3 ig((unsigned)(2 * qblocks(a.d) * a.k));
        if (dtype == MC_DTYPE_F64)
            hipLaunchKernelGGL(gmm_invert<double>, ig, dim3(kQB), inv_lds, stream, a);
        else
            hipLaunchKernelGGL(gmm_invert<float>, ig, dim3(kQB), inv_lds, stream, a);
    }
    const void* f = dtype == MC_DTYPE_F64 ? reinterpret_cast<const void*>(&gmm_items<double>)
                                          : reinterpret_cast<const void*>(&gmm_items<float>);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return note_hip_error(e);
    }
    if (dtype == MC_DTYPE_F64)
        hipLaunchKernelGGL(gmm_items<double>, dim3((unsigned)grid), dim3(kQB), lds, stream, a);
    else
        hipLaunchKernelGGL(gmm_items<float>, dim3((unsigned)grid), dim3(kQB), lds, stream, a);
    hipLaunchKernelGGL(gmm_points, dim3((unsigned)pblocks), dim3(kQB), 0, stream, a);
    if (a.total)
        hipLaunchKernelGGL(gmm_total, dim3(1), dim3(kQB), 0, stream, a.partial, pblocks,
                           a.total);
    return note_hip_error(hipGetLastError());
}

} // namespace mc
