// mc_api.hip -- the C ABI (include/mc.h): argument checks on the host,
// workspace carving, and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <atomic>
#include <vector>

#include "mc.h"
#include "mc_batched.h"
#include "mc_batched_bwd.h"
#include "mc_gmm.h"
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

namespace {
__global__ void copy_i32_kernel(int32_t* __restrict__ dst,
                                const int* __restrict__ src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
} // namespace

hipError_t launch_copy_i32(int32_t* dst, const int* src, int64_t n,
                           hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(copy_i32_kernel, dim3(blocks), dim3(256), 0, stream, dst,
                       src, n);
    return hipGetLastError();
}

// ------------------------------------------------------------ last error
static thread_local hipError_t g_last_hip = hipSuccess;

hipError_t note_hip_error(hipError_t e)
{
    if (e != hipSuccess) g_last_hip = e;
    return e;
}

// ------------------------------------------------------------- profiling
namespace {

constexpr int kMaxProfPairs = 4096;

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> begin, end; // created lazily, reused
    std::vector<int> kind;
    int used = 0;
    int64_t launches[2] = {0, 0};
    double bytes[2] = {0.0, 0.0}, flops[2] = {0.0, 0.0};
};

Profiler g_prof;

} // namespace

ProfMark prof_begin(hipStream_t stream, int kind)
{
    ProfMark m;
    m.kind = kind == MC_PROF_PANEL ? MC_PROF_PANEL : MC_PROF_UPDATE;
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
        g_prof.kind.push_back(0);
    }
    if (hipEventRecord(g_prof.begin[i], stream) != hipSuccess) return m;
    g_prof.kind[i] = m.kind;
    g_prof.used = i + 1;
    m.slot = i;
    return m;
}

void prof_end(hipStream_t stream, ProfMark m, int64_t launches,
              double alg_bytes, double alg_flops)
{
    if (!g_prof.on) return;
    g_prof.launches[m.kind] += launches;
    g_prof.bytes[m.kind] += alg_bytes;
    g_prof.flops[m.kind] += alg_flops;
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
    w.piv_col = nullptr;
    w.state = reinterpret_cast<DevState*>(p);
    return w;
}

// ------------------------------------------------------------- blocked path
static int64_t blocked_ldw(int64_t n, size_t elem)
{
    const int64_t per = 128 / (int64_t)elem; // 128-byte rows
    return (n + per - 1) / per * per;
}

static size_t blocked_bytes(int64_t n, int dtype, int64_t b, bool with_w)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t ldw = blocked_ldw(n, elem);
    size_t t = 0;
    if (with_w) t += align_up(elem * (size_t)n * (size_t)ldw, kAlign); // W
    t += align_up(elem * (size_t)n * (size_t)b, kAlign);       // L
    t += align_up(sizeof(int) * (size_t)n, kAlign);            // piv_pos
    t += align_up(sizeof(double) * (size_t)n, kAlign);         // piv_val
    t += 4 * align_up(sizeof(int) * (size_t)n, kAlign);        // perm, perm0, colsrc x2
    t += 4 * align_up(sizeof(int) * (size_t)kMaxPanel, kAlign); // srcp, moved x2
    t += align_up(elem * (size_t)kMaxPanel * 16, kAlign);       // dinv
    t += align_up(sizeof(int) * (size_t)kMaxPanel, kAlign);     // stepflag
    t += align_up(3 * sizeof(int), kAlign);                     // claim
    t += align_up(sizeof(unsigned long long) * 4 * kSplitSlices, kAlign); // xrec
    t += align_up(elem * 2 * kSplitSlices * (size_t)kMaxPanel, kAlign);  // xcol
    t += align_up(sizeof(DevState), kAlign);
    return t;
}

size_t blocked_workspace_bytes(int64_t n, int dtype, int64_t b)
{
    return blocked_bytes(n, dtype, b, true);
}

template <typename T>
BlkWork<T> blocked_carve(void* work, int64_t n, int64_t b, bool with_w)
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
    w.W = with_w ? reinterpret_cast<T*>(take(sizeof(T) * (size_t)n * (size_t)ldw))
                 : nullptr;
    w.ldl = b;
    w.L = reinterpret_cast<T*>(take(sizeof(T) * (size_t)n * (size_t)b));
    w.piv_pos = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.piv_val = reinterpret_cast<double*>(take(sizeof(double) * (size_t)n));
    w.perm = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.perm0 = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.colsrc = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.srcp = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.moved = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.colsrc_b = reinterpret_cast<int*>(take(sizeof(int) * (size_t)n));
    w.srcp_b = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.moved_b = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.dinv = reinterpret_cast<T*>(take(sizeof(T) * (size_t)kMaxPanel * 16));
    w.stepflag = reinterpret_cast<int*>(take(sizeof(int) * (size_t)kMaxPanel));
    w.claim = reinterpret_cast<int*>(take(3 * sizeof(int)));
    w.xrec = reinterpret_cast<unsigned long long*>(
        take(sizeof(unsigned long long) * 4 * kSplitSlices));
    w.xcol = reinterpret_cast<T*>(take(sizeof(T) * 2 * kSplitSlices * (size_t)kMaxPanel));
    w.state = reinterpret_cast<DevState*>(take(sizeof(DevState)));
    return w;
}

template BlkWork<double> blocked_carve<double>(void*, int64_t, int64_t, bool);
template BlkWork<float> blocked_carve<float>(void*, int64_t, int64_t, bool);

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
    case MC_ERR_TOO_LARGE:
        return "matrix too large for the library's fixed scratch array (MC_NOALLOC_BYTES)";
    default: break;
    }
    if (status < 0 && status > -20) return "invalid argument";
    return "unknown status";
}

extern "C" const char* mc_last_hip_error(void)
{
    return hipGetErrorString(g_last_hip);
}

static std::atomic<bool> g_lookahead_on{true};

extern "C" int mc_lookahead_enable(int on)
{
    return g_lookahead_on.exchange(on != 0) ? 1 : 0;
}

extern "C" int mc_split_panel_enable(int on) { return split_panel_set(on); }

extern "C" int mc_batched_spare_xcd0(int on) { return batched_spare_xcc0(on); }

extern "C" mc_status mc_profile_enable(int on)
{
    g_prof.on = on != 0;
    if (g_prof.on) {
        g_prof.used = 0;
        for (int k = 0; k < 2; ++k) {
            g_prof.launches[k] = 0;
            g_prof.bytes[k] = g_prof.flops[k] = 0.0;
        }
    }
    return MC_OK;
}

extern "C" mc_status mc_profile_read(int kind, double* elapsed_ms,
                                     int64_t* launches, double* alg_bytes,
                                     double* alg_flops)
{
    if (kind != MC_PROF_UPDATE && kind != MC_PROF_PANEL) return -1;
    double total = 0.0;
    for (int i = 0; i < g_prof.used; ++i) {
        if (g_prof.kind[i] != kind) continue;
        if (hipEventSynchronize(g_prof.end[i]) != hipSuccess) return MC_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_prof.begin[i], g_prof.end[i]) !=
            hipSuccess)
            return MC_ERR_HIP;
        total += ms;
    }
    if (elapsed_ms) *elapsed_ms = total;
    if (launches) *launches = g_prof.launches[kind];
    if (alg_bytes) *alg_bytes = g_prof.bytes[kind];
    if (alg_flops) *alg_flops = g_prof.flops[kind];
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

extern "C" int64_t mc_default_panel(int64_t n, int dtype)
{
    return n < 0 ? 0 : default_panel(n, dtype);
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

// ------------------------------------------------------------- batched path

static TuneTable default_table(int dtype)
{
    TuneTable t;
    const int64_t b64[kTuneBuckets] = {16, 32, 32, 64, 64, 64};
    const int64_t b32[kTuneBuckets] = {16, 32, 64, 64, 64, 64};
    const int tile[kTuneBuckets] = {32, 32, 64, 64, 64, 64};
    for (int k = 0; k < kTuneBuckets; ++k) {
        t.b[k] = dtype == MC_DTYPE_F64 ? b64[k] : b32[k];
        t.tile[k] = tile[k];
    }
    return t;
}

static bool g_tune_init = false;
static TuneTable g_tune[2][3]; // [dtype][update]

static TuneTable& tune_table(int dtype, int update)
{
    if (!g_tune_init) {
        for (int d = 0; d < 2; ++d)
            for (int u = 0; u < 3; ++u) g_tune[d][u] = default_table(d);
        g_tune_init = true;
    }
    return g_tune[dtype][update];
}

static bool batched_supported(int dtype, int update)
{
    if (dtype == MC_DTYPE_F64) return update == MC_UPDATE_NATIVE;
    return dtype == MC_DTYPE_F32 &&
           (update == MC_UPDATE_NATIVE || update == MC_UPDATE_F32 ||
            update == MC_UPDATE_BF16X3);
}

static TuneTable effective_table(int dtype, int update, int64_t b)
{
    TuneTable t = tune_table(dtype, update);
    if (b > 0)
        for (int k = 0; k < kTuneBuckets; ++k) t.b[k] = b;
    return t;
}

static size_t batched_header_bytes(int64_t batch)
{
    return align_up(sizeof(int) * 64, 256) + align_up(sizeof(int) * (size_t)std::max<int64_t>(batch, 1), 256);
}

extern "C" size_t mc_logdet_batched_workspace(int64_t batch, int64_t n_max,
                                              int dtype, int update, int64_t b)
{
    if (batch < 0 || n_max < 0 || n_max > kMaxN || b == 0 || b > kMaxPanel)
        return 0;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return 0;
    if (update < 0 || update > 2 || !batched_supported(dtype, update)) return 0;
    const TuneTable t = effective_table(dtype, update, b);
    return batched_header_bytes(batch) +
           (size_t)batch * batched_region_bytes(n_max, dtype, t);
}

static mc_status batched_call(const void* const* A_array, const int64_t* n_array,
                              const int64_t* lda_array, int64_t batch,
                              int64_t n_max, int dtype, int update,
                              const TuneTable& t, mc_result* out, void* work,
                              size_t work_bytes, hipStream_t st,
                              int32_t* const* perm_array = nullptr)
{
    const bool with_w = perm_array == nullptr;
    const size_t need = batched_header_bytes(batch) +
                        (size_t)batch * batched_region_bytes(n_max, dtype, t, with_w);
    if (work_bytes < need) return MC_ERR_WORKSPACE;
    BatchArgs a;
    a.A_array = A_array;
    a.n_array = n_array;
    a.lda_array = lda_array;
    a.batch = batch;
    a.n_max = n_max;
    a.update = update;
    a.table = t;
    unsigned char* base = static_cast<unsigned char*>(work);
    a.counter = reinterpret_cast<int*>(base);
    a.order = reinterpret_cast<int*>(base + align_up(sizeof(int) * 64, 256));
    a.regions = base + batched_header_bytes(batch);
    a.region_stride = batched_region_bytes(n_max, dtype, t, with_w);
    a.out = out;
    a.perm_array = perm_array;
    a.skip_xcc0 = batched_spare_xcc0_on() ? 1 : 0;
    const hipError_t e = launch_batched(a, dtype, batched_lds_bytes(dtype, t), st);
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

extern "C" mc_status mc_logdet_batched(const void* const* A_array,
                                       const int64_t* n_array,
                                       const int64_t* lda_array, int64_t batch,
                                       int64_t n_max, int dtype, int update,
                                       int64_t b, mc_result* out, void* work,
                                       size_t work_bytes, void* stream)
{
    if (batch < 0) return -4;
    if (batch > 0 && (A_array == nullptr)) return -1;
    if (batch > 0 && (n_array == nullptr)) return -2;
    if (batch > 0 && (lda_array == nullptr)) return -3;
    if (n_max < 0 || n_max > kMaxN) return -5;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -6;
    if (update < MC_UPDATE_NATIVE || update > MC_UPDATE_BF16X3) return -7;
    if (b == 0 || b > kMaxPanel) return -8;
    if (!batched_supported(dtype, update)) return MC_ERR_UNSUPPORTED;
    if (batch > 0 && out == nullptr) return -9;
    if (batch == 0) return MC_OK;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -10;
    return batched_call(A_array, n_array, lda_array, batch, n_max, dtype,
                        update, effective_table(dtype, update, b), out, work,
                        work_bytes, static_cast<hipStream_t>(stream));
}

extern "C" size_t mc_logdet_batched_factor_workspace(int64_t batch, int64_t n_max,
                                                     int dtype, int update, int64_t b)
{
    if (batch < 0 || n_max < 0 || n_max > kMaxN || b == 0 || b > kMaxPanel)
        return 0;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return 0;
    if (update < 0 || update > 2 || !batched_supported(dtype, update)) return 0;
    const TuneTable t = effective_table(dtype, update, b);
    return batched_header_bytes(batch) +
           (size_t)batch * batched_region_bytes(n_max, dtype, t, false);
}

extern "C" mc_status mc_logdet_batched_factor(void* const* A_array, const int64_t* n_array,
                                              const int64_t* lda_array,
                                              int32_t* const* perm_array, int64_t batch,
                                              int64_t n_max, int dtype, int update,
                                              int64_t b, mc_result* out, void* work,
                                              size_t work_bytes, void* stream)
{
    if (batch < 0) return -5;
    if (batch > 0 && A_array == nullptr) return -1;
    if (batch > 0 && n_array == nullptr) return -2;
    if (batch > 0 && lda_array == nullptr) return -3;
    if (batch > 0 && perm_array == nullptr) return -4;
    if (n_max < 0 || n_max > kMaxN) return -6;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -7;
    if (update < MC_UPDATE_NATIVE || update > MC_UPDATE_BF16X3) return -8;
    if (b == 0 || b > kMaxPanel) return -9;
    if (!batched_supported(dtype, update)) return MC_ERR_UNSUPPORTED;
    if (batch > 0 && out == nullptr) return -10;
    if (batch == 0) return MC_OK;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -11;
    return batched_call(reinterpret_cast<const void* const*>(A_array), n_array, lda_array,
                        batch, n_max, dtype, update, effective_table(dtype, update, b),
                        out, work, work_bytes, static_cast<hipStream_t>(stream),
                        perm_array);
}

// Largest n_max of the batched backward (its row permutation stages one
// row in LDS).
static constexpr int64_t kBatchedBwdMaxN = 16384;

extern "C" size_t mc_logdet_batched_backward_workspace(int64_t batch, int64_t n_max,
                                                      int dtype)
{
    if (batch < 0 || n_max < 0 || n_max > kBatchedBwdMaxN) return 0;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return 0;
    return batched_bwd_workspace_bytes(batch, n_max, dtype);
}

extern "C" mc_status mc_logdet_batched_backward(
    const void* const* LU_array, const int64_t* n_array, const int64_t* ld_array,
    const int32_t* const* perm_array, int64_t batch, int64_t n_max, int dtype,
    const double* grad_out, const mc_result* fwd, void* const* G_array,
    const int64_t* ldg_array, void* work, size_t work_bytes, void* stream)
{
    if (batch < 0) return -5;
    if (batch > 0 && LU_array == nullptr) return -1;
    if (batch > 0 && n_array == nullptr) return -2;
    if (batch > 0 && ld_array == nullptr) return -3;
    if (batch > 0 && perm_array == nullptr) return -4;
    if (n_max < 0 || n_max > kBatchedBwdMaxN) return -6;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -7;
    if (batch > 0 && G_array == nullptr) return -10;
    if (batch > 0 && ldg_array == nullptr) return -11;
    if (batch == 0) return MC_OK;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -12;
    if (work_bytes < batched_bwd_workspace_bytes(batch, n_max, dtype)) return MC_ERR_WORKSPACE;
    BatchedBwdArgs a{};
    a.LU_array = LU_array;
    a.n_array = n_array;
    a.ld_array = ld_array;
    a.perm_array = perm_array;
    a.batch = batch;
    a.n_max = n_max;
    a.grad_out = grad_out;
    a.fwd = fwd;
    a.G_array = G_array;
    a.ldg_array = ldg_array;
    const hipError_t e = launch_batched_backward(a, dtype, work,
                                                 static_cast<hipStream_t>(stream));
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

extern "C" mc_status mc_tune_get(int dtype, int update, int64_t* b, int* tile)
{
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -1;
    if (update < 0 || update > 2) return -2;
    const TuneTable& t = tune_table(dtype, update);
    for (int k = 0; k < kTuneBuckets; ++k) {
        if (b) b[k] = t.b[k];
        if (tile) tile[k] = t.tile[k];
    }
    return MC_OK;
}

extern "C" mc_status mc_tune_set(int dtype, int update, const int64_t* b,
                                 const int* tile)
{
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -1;
    if (update < 0 || update > 2) return -2;
    if (!b) return -3;
    if (!tile) return -4;
    for (int k = 0; k < kTuneBuckets; ++k) {
        if (b[k] < 1 || b[k] > kMaxPanel) return -3;
        if (tile[k] != 32 && tile[k] != 64) return -4;
    }
    TuneTable& t = tune_table(dtype, update);
    for (int k = 0; k < kTuneBuckets; ++k) {
        t.b[k] = b[k];
        t.tile[k] = tile[k];
    }
    return MC_OK;
}

// --- autotuner: synthetic batches per bucket, candidates timed with events
namespace {

constexpr int kTuneReps = 2;
constexpr int64_t kTuneCandB[] = {16, 32, 64, 128};
constexpr int kTuneCandTile[] = {32, 64};

int64_t tune_size(int k, int64_t n_max_tune)
{
    if (k < kTuneBuckets - 1) return std::min<int64_t>(tune_bucket_max(k), n_max_tune);
    return n_max_tune > tune_bucket_max(kTuneBuckets - 2) ? n_max_tune : 0;
}

int64_t tune_count(int64_t n, int elem)
{
    const double bytes = (double)elem * n * n;
    const int64_t cap = (int64_t)(1.0e9 / std::max(bytes, 1.0));
    return std::max<int64_t>(8, std::min<int64_t>(512, cap));
}

template <typename T>
__global__ void tune_fill(T* A, int64_t n, int64_t count, uint32_t seed)
{
    const int64_t total = n * n * count;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = e / (n * n), r = e % (n * n), i = r / n, j = r % n;
        uint32_t h = (uint32_t)(e * 2654435761u) ^ seed;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        const double u = (double)(h & 0xffffff) / 16777216.0 * 2.0 - 1.0;
        A[e] = (T)(u + (i == j ? (double)n : 0.0));
        (void)m;
    }
}

__global__ void tune_meta(const unsigned char* base, size_t elem, int64_t n,
                          int64_t count, const void** ptrs, int64_t* ns,
                          int64_t* ldas)
{
    for (int64_t k = threadIdx.x; k < count; k += blockDim.x) {
        ptrs[k] = base + (size_t)k * n * n * elem;
        ns[k] = n;
        ldas[k] = n;
    }
}

size_t tune_bytes(int dtype, int64_t n, const TuneTable& worst)
{
    const int elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t count = tune_count(n, elem);
    size_t t = align_up((size_t)elem * n * n * count, 256);
    t += 3 * align_up(sizeof(int64_t) * count, 256);
    t += align_up(sizeof(mc_result) * count, 256);
    t += batched_header_bytes(count) + (size_t)count * batched_region_bytes(n, dtype, worst);
    return t;
}

TuneTable worst_table()
{
    TuneTable t;
    for (int k = 0; k < kTuneBuckets; ++k) {
        t.b[k] = kMaxPanel;
        t.tile[k] = 64;
    }
    return t;
}

} // namespace

extern "C" size_t mc_autotune_workspace(int dtype, int64_t n_max_tune)
{
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return 0;
    if (n_max_tune < 1 || n_max_tune > 4096) return 0;
    size_t best = 0;
    for (int k = 0; k < kTuneBuckets; ++k) {
        const int64_t n = tune_size(k, n_max_tune);
        if (n > 0) best = std::max(best, tune_bytes(dtype, n, worst_table()));
    }
    return best;
}

extern "C" mc_status mc_autotune_batched(int dtype, int update,
                                         int64_t n_max_tune, void* work,
                                         size_t work_bytes, void* stream)
{
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -1;
    if (update < 0 || update > 2) return -2;
    if (!batched_supported(dtype, update)) return MC_ERR_UNSUPPORTED;
    if (n_max_tune < 1 || n_max_tune > 4096) return -3;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -4;
    if (work_bytes < mc_autotune_workspace(dtype, n_max_tune)) return MC_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    TuneTable& table = tune_table(dtype, update);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MC_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MC_ERR_HIP;
    }
    mc_status rc = MC_OK;
    for (int k = 0; k < kTuneBuckets && rc == MC_OK; ++k) {
        const int64_t n = tune_size(k, n_max_tune);
        if (n <= 0) continue;
        const int64_t count = tune_count(n, elem);
        unsigned char* p = static_cast<unsigned char*>(work);
        unsigned char* mats = p;
        p += align_up((size_t)elem * n * n * count, 256);
        const void** ptrs = reinterpret_cast<const void**>(p);
        p += align_up(sizeof(int64_t) * count, 256);
        int64_t* ns = reinterpret_cast<int64_t*>(p);
        p += align_up(sizeof(int64_t) * count, 256);
        int64_t* ldas = reinterpret_cast<int64_t*>(p);
        p += align_up(sizeof(int64_t) * count, 256);
        mc_result* outs = reinterpret_cast<mc_result*>(p);
        p += align_up(sizeof(mc_result) * count, 256);
        const size_t rest = work_bytes - (size_t)(p - static_cast<unsigned char*>(work));
        if (dtype == MC_DTYPE_F64)
            hipLaunchKernelGGL(tune_fill<double>, dim3(1024), dim3(256), 0, st,
                               reinterpret_cast<double*>(mats), n, count, 12345u + k);
        else
            hipLaunchKernelGGL(tune_fill<float>, dim3(1024), dim3(256), 0, st,
                               reinterpret_cast<float*>(mats), n, count, 12345u + k);
        hipLaunchKernelGGL(tune_meta, dim3(1), dim3(256), 0, st, mats, (size_t)elem, n,
                           count, ptrs, ns, ldas);
        float best_ms = 1e30f;
        int64_t best_b = table.b[k];
        int best_tile = table.tile[k];
        for (int64_t cb : kTuneCandB) {
            if (cb > n && cb != kTuneCandB[0]) continue;
            for (int ct : kTuneCandTile) {
                TuneTable t = table;
                t.b[k] = cb;
                t.tile[k] = ct;
                mc_status s1 = batched_call(ptrs, ns, ldas, count, n, dtype, update, t,
                                            outs, p, rest, st);
                if (s1 != MC_OK) { rc = s1; break; }
                if (hipEventRecord(e0, st) != hipSuccess) { rc = MC_ERR_HIP; break; }
                for (int r = 0; r < kTuneReps && rc == MC_OK; ++r)
                    rc = batched_call(ptrs, ns, ldas, count, n, dtype, update, t, outs,
                                      p, rest, st);
                if (rc != MC_OK) break;
                if (hipEventRecord(e1, st) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess) { rc = MC_ERR_HIP; break; }
                float ms = 0;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = MC_ERR_HIP; break; }
                if (ms < best_ms) {
                    best_ms = ms;
                    best_b = cb;
                    best_tile = ct;
                }
            }
            if (rc != MC_OK) break;
        }
        if (rc == MC_OK) {
            table.b[k] = best_b;
            table.tile[k] = best_tile;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// ------------------------------------------------------ factor / backward

extern "C" size_t mc_logdet_factor_workspace(int64_t n, int dtype, int update,
                                             int64_t b)
{
    if (n < 0 || n > kMaxN) return 0;
    if (b < 0) b = default_panel(n, dtype);
    if (!blocked_supported(dtype, update, b)) return 0;
    return blocked_bytes(n, dtype, b, false);
}

extern "C" mc_status mc_logdet_factor(void* A, int64_t n, int64_t lda,
                                      int dtype, int update, int64_t b,
                                      int32_t* perm, mc_result* out,
                                      void* work, size_t work_bytes,
                                      void* stream)
{
    if (n < 0 || n > kMaxN) return -2;
    if (n > 0 && A == nullptr) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -4;
    if (update < MC_UPDATE_NATIVE || update > MC_UPDATE_BF16X3) return -5;
    if (b < 0) b = default_panel(n, dtype);
    if (!blocked_supported(dtype, update, b)) return MC_ERR_UNSUPPORTED;
    if (n > 0 && perm == nullptr) return -7;
    if (out == nullptr) return -8;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0)
        return launch_write_result(out, 0.0, 1.0, 0, st) == hipSuccess ? MC_OK
                                                                       : MC_ERR_HIP;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -9;
    if (work_bytes < blocked_bytes(n, dtype, b, false)) return MC_ERR_WORKSPACE;
    hipError_t e;
    if (dtype == MC_DTYPE_F64) {
        BlkWork<double> w = blocked_carve<double>(work, n, b, false);
        w.W = static_cast<double*>(A);
        w.ldw = lda;
        w.perm = perm;
        e = launch_blocked<double>(w.W, n, lda, b, update, w, out, st, true,
                                   g_lookahead_on.load());
    } else {
        BlkWork<float> w = blocked_carve<float>(work, n, b, false);
        w.W = static_cast<float*>(A);
        w.ldw = lda;
        w.perm = perm;
        e = launch_blocked<float>(w.W, n, lda, b, update, w, out, st, true,
                                  g_lookahead_on.load());
    }
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

extern "C" size_t mc_logdet_backward_workspace(int64_t n, int dtype)
{
    if (n < 0 || n > kMaxN) return 0;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return 0;
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t ldz = blocked_ldw(n, elem);
    return align_up(elem * (size_t)n * (size_t)ldz, kAlign) +
           align_up(sizeof(int) * (size_t)std::max<int64_t>(n, 1), kAlign) +
           align_up(sizeof(DevState), kAlign);
}

static mc_status backward_impl(const void* LU, int64_t n, int64_t ld,
                               const int32_t* perm, int dtype,
                               const double* grad_out, const mc_result* fwd,
                               void* gradA, int64_t ldg, void* work,
                               hipStream_t st)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    const int64_t ldz = blocked_ldw(n, elem);
    char* p = static_cast<char*>(work);
    void* Z = p;
    p += align_up(elem * (size_t)n * (size_t)ldz, kAlign);
    int* ident = reinterpret_cast<int*>(p);
    p += align_up(sizeof(int) * (size_t)n, kAlign);
    DevState* state = reinterpret_cast<DevState*>(p);
    hipError_t e;
    if (dtype == MC_DTYPE_F64)
        e = launch_backward<double>(static_cast<const double*>(LU), ld, perm, n,
                                    grad_out, fwd, static_cast<double*>(gradA), ldg,
                                    BwdWork<double>{static_cast<double*>(Z), ldz,
                                                    ident, state},
                                    st);
    else
        e = launch_backward<float>(static_cast<const float*>(LU), ld, perm, n,
                                   grad_out, fwd, static_cast<float*>(gradA), ldg,
                                   BwdWork<float>{static_cast<float*>(Z), ldz,
                                                  ident, state},
                                   st);
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

extern "C" mc_status mc_logdet_backward(const void* LU, int64_t n, int64_t ld,
                                        const int32_t* perm, int dtype,
                                        const double* grad_out,
                                        const mc_result* fwd, void* gradA,
                                        int64_t ldg, void* work,
                                        size_t work_bytes, void* stream)
{
    if (n < 0 || n > kMaxN) return -2;
    if (n > 0 && LU == nullptr) return -1;
    if (ld < (n > 1 ? n : 1)) return -3;
    if (n > 0 && perm == nullptr) return -4;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -5;
    if (n > 0 && gradA == nullptr) return -8;
    if (ldg < (n > 1 ? n : 1)) return -9;
    if (n == 0) return MC_OK;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -10;
    if (work_bytes < mc_logdet_backward_workspace(n, dtype)) return MC_ERR_WORKSPACE;
    return backward_impl(LU, n, ld, perm, dtype, grad_out, fwd, gradA, ldg, work,
                         static_cast<hipStream_t>(stream));
}

// ---- backward with the factors recomputed: a copy of A is factored in the
// workspace, then the backward runs on it.  Layout: LU (n x ldw), perm,
// the forward result, then one region shared by the factor call's
// workspace and the backward's (the second starts after the first ends on
// the stream).
namespace {

template <typename T>
__global__ void copy_matrix_kernel(const T* __restrict__ A, int64_t lda,
                                   T* __restrict__ B, int64_t ldb, int64_t n)
{
    const int64_t i = blockIdx.x;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) B[i * ldb + j] = A[i * lda + j];
}

struct RecomputeLayout {
    size_t lu, perm, res, region, total;
    int64_t ldw;
};

RecomputeLayout recompute_layout(int64_t n, int dtype, int64_t b)
{
    const size_t elem = dtype == MC_DTYPE_F64 ? 8 : 4;
    RecomputeLayout L;
    L.ldw = blocked_ldw(n, elem);
    L.lu = 0;
    L.perm = L.lu + align_up(elem * (size_t)n * (size_t)L.ldw, kAlign);
    L.res = L.perm + align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1), kAlign);
    L.region = L.res + align_up(sizeof(mc_result), kAlign);
    L.total = L.region + std::max(blocked_bytes(n, dtype, b, false),
                                  mc_logdet_backward_workspace(n, dtype));
    return L;
}

} // namespace

extern "C" size_t mc_logdet_backward_recompute_workspace(int64_t n, int dtype,
                                                         int update, int64_t b)
{
    if (n < 0 || n > kMaxN) return 0;
    if (b < 0) b = default_panel(n, dtype);
    if (!blocked_supported(dtype, update, b)) return 0;
    return recompute_layout(n, dtype, b).total;
}

extern "C" mc_status mc_logdet_backward_recompute(
    const void* A, int64_t n, int64_t lda, int dtype, int update, int64_t b,
    const double* grad_out, void* gradA, int64_t ldg, mc_result* out,
    void* work, size_t work_bytes, void* stream)
{
    if (n < 0 || n > kMaxN) return -2;
    if (n > 0 && A == nullptr) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -4;
    if (update < MC_UPDATE_NATIVE || update > MC_UPDATE_BF16X3) return -5;
    if (b < 0) b = default_panel(n, dtype);
    if (!blocked_supported(dtype, update, b)) return MC_ERR_UNSUPPORTED;
    if (n > 0 && gradA == nullptr) return -8;
    if (ldg < (n > 1 ? n : 1)) return -9;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0)
        return out == nullptr || launch_write_result(out, 0.0, 1.0, 0, st) == hipSuccess
                   ? MC_OK
                   : MC_ERR_HIP;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -11;
    const RecomputeLayout L = recompute_layout(n, dtype, b);
    if (work_bytes < L.total) return MC_ERR_WORKSPACE;
    char* base = static_cast<char*>(work);
    int32_t* perm = reinterpret_cast<int32_t*>(base + L.perm);
    mc_result* res = out ? out : reinterpret_cast<mc_result*>(base + L.res);
    void* region = base + L.region;
    hipError_t e;
    if (dtype == MC_DTYPE_F64) {
        double* LU = reinterpret_cast<double*>(base + L.lu);
        hipLaunchKernelGGL(copy_matrix_kernel<double>, dim3((unsigned)n), dim3(256), 0, st,
                           static_cast<const double*>(A), lda, LU, L.ldw, n);
        BlkWork<double> w = blocked_carve<double>(region, n, b, false);
        w.W = LU;
        w.ldw = L.ldw;
        w.perm = perm;
        e = launch_blocked<double>(LU, n, L.ldw, b, update, w, res, st, true,
                                   g_lookahead_on.load());
        if (e == hipSuccess)
            return backward_impl(LU, n, L.ldw, perm, dtype, grad_out, res, gradA, ldg,
                                 region, st);
    } else {
        float* LU = reinterpret_cast<float*>(base + L.lu);
        hipLaunchKernelGGL(copy_matrix_kernel<float>, dim3((unsigned)n), dim3(256), 0, st,
                           static_cast<const float*>(A), lda, LU, L.ldw, n);
        BlkWork<float> w = blocked_carve<float>(region, n, b, false);
        w.W = LU;
        w.ldw = L.ldw;
        w.perm = perm;
        e = launch_blocked<float>(LU, n, L.ldw, b, update, w, res, st, true,
                                  g_lookahead_on.load());
        if (e == hipSuccess)
            return backward_impl(LU, n, L.ldw, perm, dtype, grad_out, res, gradA, ldg,
                                 region, st);
    }
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

// `shared`: the call may use the device's scheduling state (lookahead's
// side stream, the ordering of blocked calls); false keeps every kernel on
// `stream` and creates no runtime object.
static mc_status logdet_impl(const void* A, int64_t n, int64_t lda, int dtype,
                             int update, int64_t b, int32_t* piv_col,
                             mc_result* out, void* work, size_t work_bytes,
                             void* stream, bool shared = true)
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
        PlainWork w = plain_carve(work, n);
        w.piv_col = piv_col;
        e = launch_plain_f64(static_cast<const double*>(A), n, lda, w, out, st);
    } else {
        if (work_bytes < blocked_workspace_bytes(n, dtype, b))
            return MC_ERR_WORKSPACE;
        if (dtype == MC_DTYPE_F64) {
            const BlkWork<double> w = blocked_carve<double>(work, n, b);
            e = launch_blocked<double>(static_cast<const double*>(A), n, lda,
                                       b, update, w, out, st, false,
                                       shared && g_lookahead_on.load(), shared);
            // after the last panel, position s holds the column step s took
            if (e == hipSuccess && piv_col) e = launch_copy_i32(piv_col, w.perm, n, st);
        } else {
            const BlkWork<float> w = blocked_carve<float>(work, n, b);
            e = launch_blocked<float>(static_cast<const float*>(A), n, lda, b,
                                      update, w, out, st, false,
                                      shared && g_lookahead_on.load(), shared);
            if (e == hipSuccess && piv_col) e = launch_copy_i32(piv_col, w.perm, n, st);
        }
    }
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

namespace mc {
mc_status logdet_fixed_work(const void* A, int64_t n, int64_t lda, int dtype,
                            int update, int64_t b, mc_result* out, void* work,
                            size_t work_bytes, void* stream)
{
    return logdet_impl(A, n, lda, dtype, update, b, nullptr, out, work,
                       work_bytes, stream, false);
}
} // namespace mc

extern "C" mc_status mc_logdet(const void* A, int64_t n, int64_t lda,
                               int dtype, int update, int64_t b,
                               mc_result* out, void* work, size_t work_bytes,
                               void* stream)
{
    return logdet_impl(A, n, lda, dtype, update, b, nullptr, out, work,
                       work_bytes, stream);
}

extern "C" mc_status mc_logdet_pivots(const void* A, int64_t n, int64_t lda,
                                      int dtype, int update, int64_t b,
                                      int32_t* piv_col, mc_result* out,
                                      void* work, size_t work_bytes,
                                      void* stream)
{
    if (n > 0 && piv_col == nullptr) return -7;
    const mc_status s = logdet_impl(A, n, lda, dtype, update, b, piv_col, out,
                                    work, work_bytes, stream);
    // logdet_impl numbers `out` as argument 7; here it is argument 8
    return s == -7 ? -8 : (s == -8 ? -9 : s);
}

extern "C" mc_status mc_logdet_rule(const void* A, int64_t n, int64_t lda,
                                    int rule, int32_t* piv_col, mc_result* out,
                                    void* work, size_t work_bytes, void* stream)
{
    if (n < 0 || n > kMaxN) return -2;
    if (n > 0 && A == nullptr) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (rule < MC_PIVOT_MAXABS || rule > MC_PIVOT_CLOSEST_TO_ONE) return -4;
    if (out == nullptr) return -6;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0)
        return launch_write_result(out, 0.0, 1.0, 0, st) == hipSuccess ? MC_OK
                                                                       : MC_ERR_HIP;
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -7;
    if (work_bytes < plain_workspace_bytes(n)) return MC_ERR_WORKSPACE;
    PlainWork w = plain_carve(work, n);
    w.piv_col = piv_col;
    const hipError_t e =
        launch_plain_f64(static_cast<const double*>(A), n, lda, w, out, st, rule);
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}

// ------------------------------------------------------ mixture log-likelihood

// Largest dimension of the mixture call (the right-hand sides of one work
// item are kept in the workspace, 64 x d).
static constexpr int64_t kGmmMaxD = 16384;

extern "C" size_t mc_gmm_loglik_workspace(int64_t m, int64_t d, int64_t k, int dtype)
{
    if (m < 0 || d < 1 || d > kGmmMaxD || k < 1 || k > (1 << 20)) return 0;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return 0;
    return gmm_workspace_bytes(m, d, k, dtype);
}

extern "C" mc_status mc_gmm_loglik(const void* X, int64_t m, int64_t d, int64_t ldx,
                                   const void* means, int64_t ldmu, int64_t k,
                                   const double* log_weights,
                                   const void* const* LU_array, const int64_t* ld_array,
                                   const int32_t* const* perm_array,
                                   const mc_result* fwd, int dtype, double* loglik,
                                   double* total, void* work, size_t work_bytes,
                                   void* stream)
{
    if (m < 0) return -2;
    if (m > 0 && X == nullptr) return -1;
    if (d < 1 || d > kGmmMaxD) return -3;
    if (ldx < d) return -4;
    if (means == nullptr) return -5;
    if (ldmu < d) return -6;
    if (k < 1 || k > (1 << 20)) return -7;
    if (log_weights == nullptr) return -8;
    if (LU_array == nullptr) return -9;
    if (ld_array == nullptr) return -10;
    if (perm_array == nullptr) return -11;
    if (fwd == nullptr) return -12;
    if (dtype != MC_DTYPE_F64 && dtype != MC_DTYPE_F32) return -13;
    if (m > 0 && loglik == nullptr) return -14;
    if (m == 0 && total == nullptr) return MC_OK;  // nothing to write
    if (work == nullptr || reinterpret_cast<uintptr_t>(work) % 256 != 0) return -16;
    if (work_bytes < gmm_workspace_bytes(m, d, k, dtype)) return MC_ERR_WORKSPACE;
    GmmArgs a{};
    a.X = X;
    a.m = m;
    a.d = d;
    a.ldx = ldx;
    a.means = means;
    a.ldmu = ldmu;
    a.k = k;
    a.log_weights = log_weights;
    a.LU_array = LU_array;
    a.ld_array = ld_array;
    a.perm_array = perm_array;
    a.fwd = fwd;
    a.loglik = loglik;
    a.total = total;
    const hipError_t e = launch_gmm(a, dtype, work, work_bytes, static_cast<hipStream_t>(stream));
    return note_hip_error(e) == hipSuccess ? MC_OK : MC_ERR_HIP;
}
