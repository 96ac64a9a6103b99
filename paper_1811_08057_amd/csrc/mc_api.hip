// mc_api.hip -- the C ABI (include/mc.h): argument checks on the host,
// workspace carving, and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "mc.h"
#include "mc_internal.h"

namespace mc {

namespace {

__global__ void write_result_kernel(mc_result* out, double logabsdet,
                                    double sign, int64_t info)
{
    out->logabsdet = logabsdet;
    out->sign = sign;
    out->info = info;
}

constexpr size_t kAlign = 256;

} // namespace

hipError_t launch_write_result(mc_result* out, double logabsdet, double sign,
                               int64_t info, hipStream_t stream)
{
    hipLaunchKernelGGL(write_result_kernel, dim3(1), dim3(1), 0, stream, out,
                       logabsdet, sign, info);
    return hipGetLastError();
}

// ------------------------------------------------------------- profiling
namespace {

constexpr int kMaxProfPairs = 4096;

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> begin, end; // created lazily, reused
    int used = 0;
    int64_t launches = 0;
    double bytes = 0.0, flops = 0.0;
};

Profiler g_prof;

} // namespace

ProfMark prof_begin(hipStream_t stream)
{
    ProfMark m;
    if (!g_prof.on || g_prof.used >= kMaxProfPairs) return m;
    const int i = g_prof.used;
    if (i >= (int)g_prof.begin.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return m;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return m;
        }
        g_prof.begin.push_back(a);
        g_prof.end.push_back(b);
    }
    if (hipEventRecord(g_prof.begin[i], stream) != hipSuccess) return m;
    g_prof.used = i + 1;
    m.slot = i;
    return m;
}

void prof_end(hipStream_t stream, ProfMark m, int64_t launches,
              double alg_bytes, double alg_flops)
{
    if (!g_prof.on) return;
    g_prof.launches += launches;
    g_prof.bytes += alg_bytes;
    g_prof.flops += alg_flops;
    if (m.slot >= 0) (void)hipEventRecord(g_prof.end[m.slot], stream);
}

static int64_t plain_ldw(int64_t n) { return (n + 15) / 16 * 16; }

size_t plain_workspace_bytes(int64_t n)
{
    const int64_t ldw = plain_ldw(n);
    size_t b = 0;
    b += align_up(sizeof(double) * (size_t)n * (size_t)ldw, kAlign); // W
    b += 2 * align_up(sizeof(double) * (size_t)ldw, kAlign);          // r
    b += align_up(sizeof(double) * (size_t)n, kAlign);                // piv_val
    b += 2 * align_up(sizeof(int) * (size_t)n, kAlign);               // slot, colid
    b += align_up(sizeof(DevState), kAlign);
    return b;
}

PlainWork plain_carve(void* work, int64_t n)
{
    const int64_t ldw = plain_ldw(n);
    char* p = static_cast<char*>(work);
    PlainWork w;
    w.ldw = ldw;
    w.W = reinterpret_cast<double*>(p);
    p += align_up(sizeof(double) * (size_t)n * (size_t)ldw, kAlign);
    for (int h = 0; h < 2; ++h) {
        w.r[h] = reinterpret_cast<double*>(p);
        p += align_up(sizeof(double) * (size_t)ldw, kAlign);
    }
    w.piv_val = reinterpret_cast<double*>(p);
    p += align_up(sizeof(double) * (size_t)n, kAlign);
    w.piv_slot = reinterpret_cast<int*>(p);
    p += align_up(sizeof(int) * (size_t)n, kAlign);
    w.colid = reinterpret_cast<int*>(p);
    p += align_up(sizeof(int) * (size_t)n, kAlign);
    w.state = reinterpret_cast<DevState*>(p);
    return w;
}

// ------------------------------------------------------------- blocked path
static int64_t blocked_ldw(int64_t n, size_t elem)
{
    const int64_t per = 128 / (int64_t)elem; // 128-byte rows
    return (n + per - 1) / per * per;
}

size_t blocked_workspace_bytes(int64_t n, int dtype, int64_t b)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t ldw = blocked_ldw(n, elem);
    size_t t = 0;
    t += align_up(elem * (size_t)n * (size_t)ldw, kAlign);     // W
    t += align_up(elem * (size_t)n * (size_t)b, kAlign);       // L
    t += align_up(sizeof(int) * (size_t)n, kAlign);            // piv_pos
    t += align_up(sizeof(double) * (size_t)n, kAlign);         // piv_val
    t += 2 * align_up(sizeof(int) * (size_t)n, kAlign);        // perm, colsrc
    t += 2 * align_up(sizeof(int) * (size_t)kMaxPanel, kAlign); // srcp, moved
    t += align_up(sizeof(DevState), kAlign);
    return t;
}

template <typename T>
BlkWork<T> blocked_carve(void* work, int64_t n, int64_t b)
{
    const int64_t ldw = blocked_ldw(n, sizeof(T));
    char* p = static_cast<char*>(work);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += align_up(bytes, kAlign);
        return q;
    };
    BlkWork<T> w;
    w.ldw = ldw;
    w.W = reinterpret_cast<T*>(take(sizeof(T) * (size_t)n * (size_t)ldw));
    w.ldl = b;
    w.L = reinterpret_cast<T*>(take(sizeof(T) * (size_t)n * (size_t)b));
    w.piv_pos = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.piv_val = reinterpret_cast<double*>(take(sizeof(double) * (size_t)n));
    w.perm = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.colsrc = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.srcp = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.moved = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.state = reinterpret_cast<DevState*>(take(sizeof(DevState)));
    return w;
}

template BlkWork<double> blocked_carve<double>(void*, int64_t, int64_t);
template BlkWork<float> blocked_carve<float>(void*, int64_t, int64_t);

} // namespace mc

using namespace mc;

// Largest n accepted: row and column indices of the kernels are 32-bit.
static constexpr int64_t kMaxN = (int64_t)1 << 30;

extern "C" int mc_version(void) { return 100; }

extern "C" const char* mc_status_string(mc_status status)
{
    switch (status) {
    case MC_OK: return "ok";
    case MC_ERR_WORKSPACE: return "workspace too small";
    case MC_ERR_HIP: return "HIP launch or query failed";
    case MC_ERR_UNSUPPORTED: return "unsupported combination of arguments";
    default: break;
    }
    if (status < 0 && status > -20) return "invalid argument";
    return "unknown status";
}

extern "C" mc_status mc_profile_enable(int on)
{
    g_prof.on = on != 0;
    if (g_prof.on) {
        g_prof.used = 0;
        g_prof.launches = 0;
        g_prof.bytes = g_prof.flops = 0.0;
    }
    return MC_OK;
}

extern "C" mc_status mc_profile_read(double* elapsed_ms, int64_t* launches,
                                     double* alg_bytes, double* alg_flops)
{
    double total = 0.0;
    for (int i = 0; i < g_prof.used; ++i) {
        if (hipEventSynchronize(g_prof.end[i]) != hipSuccess) return MC_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_prof.begin[i], g_prof.end[i]) !=
            hipSuccess)
            return MC_ERR_HIP;
        total += ms;
    }
    if (elapsed_ms) *elapsed_ms = total;
    if (launches) *launches = g_prof.launches;
    if (alg_bytes) *alg_bytes = g_prof.bytes;
    if (alg_flops) *alg_flops = g_prof.flops;
    return MC_OK;
}

static bool plain_supported(int dtype, int update, int64_t b)
{
    return b == 0 && dtype == MC_DTYPE_F64 && update == MC_UPDATE_NATIVE;
}

// Panel width for b < 0 ("library default").
static int64_t default_panel(int64_t n, int dtype)
{
    (void)dtype;
    if (n <= 256) return 32;
    if (n <= 1024) return 64;
    return 128;
}

static bool blocked_supported(int dtype, int update, int64_t b)
{
    if (b == 0 || b > kMaxPanel) return false;
    if (dtype == MC_DTYPE_F64) return update == MC_UPDATE_NATIVE;
    return dtype == MC_DTYPE_F32 &&
           (update == MC_UPDATE_NATIVE || update == MC_UPDATE_F32 ||
            update == MC_UPDATE_BF16X3);
}

extern "C" size_t mc_logdet_workspace(int64_t n, int dtype, int update,
                                      int64_t b)
{
    if (n < 0 || n > kMaxN) return 0;
    if (plain_supported(dtype, update, b)) return plain_workspace_bytes(n);
    if (b < 0) b = default_panel(n, dtype);
    if (blocked_supported(dtype, update, b))
        return blocked_workspace_bytes(n, dtype, b);
    return 0;
}

extern "C" mc_status mc_logdet(const void* A, int64_t n, int64_t lda,
                               int dtype, int update, int64_t b,
                               mc_result* out, void* work, size_t work_bytes,
                               void* stream)
{
    if (n < 0 || n > kMaxN) return -2;
    if (n > 0 && A == nullptr) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -4;
    if (update < MC_UPDATE_NATIVE || update > MC_UPDATE_BF16X3) return -5;
    if (out == nullptr) return -7;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (b < 0) b = default_panel(n, dtype);
    const bool plain = plain_supported(dtype, update, b);
    if (!plain && !blocked_supported(dtype, update, b))
        return MC_ERR_UNSUPPORTED;
    if (n == 0)
        return launch_write_result(out, 0.0, 1.0, 0, st) == hipSuccess
                   ? MC_OK
                   : MC_ERR_HIP;
    if (work == nullptr) return -8;
    if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return -8;
    hipError_t e;
    if (plain) {
        if (work_bytes < plain_workspace_bytes(n)) return MC_ERR_WORKSPACE;
        const PlainWork w = plain_carve(work, n);
        e = launch_plain_f64(static_cast<const double*>(A), n, lda, w, out, st);
    } else {
        if (work_bytes < blocked_workspace_bytes(n, dtype, b))
            return MC_ERR_WORKSPACE;
        if (dtype == MC_DTYPE_F64)
            e = launch_blocked<double>(static_cast<const double*>(A), n, lda,
                                       b, update,
                                       blocked_carve<double>(work, n, b), out,
                                       st);
        else
            e = launch_blocked<float>(static_cast<const float*>(A), n, lda, b,
                                      update, blocked_carve<float>(work, n, b),
                                      out, st);
    }
    return e == hipSuccess ? MC_OK : MC_ERR_HIP;
}
