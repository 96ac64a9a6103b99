// mc_noalloc.hip -- mc_logdet_noalloc: mc_logdet for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The workspace is a fixed device array, `scratch`, of MC_NOALLOC_BYTES,
// one copy per GPU, held until the process ends.  In host code the array's
// name is only a host-side stand-in, so its device address is looked up once
// per device with hipGetSymbolAddress (with that device current) and only
// that address is handed to the kernels.  Every call on a GPU uses the same
// array: calls that overlap on one GPU race.  The kernels initialise every
// part of the workspace they read (mc_logdet ignores its contents on
// entry), so nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "mc.h"
#include "mc_internal.h"

static __device__ __align__(256) unsigned char scratch[MC_NOALLOC_BYTES];

namespace {

constexpr int kMaxDev = 64;
std::mutex g_mu;
void* g_ptr[kMaxDev];    // device address of `scratch` on each device
bool g_looked[kMaxDev];  // lookup done (g_ptr set) on each device

// The current device's copy of `scratch`, looked up on first use.
mc_status scratch_ptr(void** out)
{
    int dev = 0;
    if (mc::note_hip_error(hipGetDevice(&dev)) != hipSuccess) return MC_ERR_HIP;
    if (dev < 0 || dev >= kMaxDev) return MC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_looked[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)mc::note_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return MC_ERR_HIP;
        }
        g_ptr[dev] = p;
        g_looked[dev] = true;
    }
    *out = g_ptr[dev];
    return MC_OK;
}

} // namespace

extern "C" mc_status mc_logdet_noalloc(const void* A, int64_t n, int64_t lda,
                                       int dtype, int update, int64_t b,
                                       mc_result* out, void* stream)
{
    // the same argument checks as mc_logdet, before anything else
    if (n < 0) return -2;
    if (n > 0 && A == nullptr) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -4;
    if (update < MC_UPDATE_NATIVE || update > MC_UPDATE_BF16X3) return -5;
    if (out == nullptr) return -7;
    const size_t need = mc_logdet_workspace(n, dtype, update, b);
    if (need == 0) return MC_ERR_UNSUPPORTED;
    if (need > (size_t)MC_NOALLOC_BYTES) return MC_ERR_TOO_LARGE;
    void* work = nullptr;
    const mc_status s = scratch_ptr(&work);
    if (s != MC_OK) return s;
    return mc::logdet_fixed_work(A, n, lda, dtype, update, b, out, work,
                                 (size_t)MC_NOALLOC_BYTES, stream);
}
