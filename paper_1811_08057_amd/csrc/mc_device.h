// mc_device.h -- device helpers shared by the condensation kernels (gfx950).
//
// Pivot search (Section 2.2): the pivot column of a row is the column of
// largest |a|, ties resolved to the smallest ORIGINAL column index so that
// the choice does not depend on where a column currently sits in memory.
// A NaN or Inf never wins; it raises the non-finite flag instead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

namespace mc {

constexpr int kWave = 64;

// Status codes kept in device memory by a running factorisation.
enum : int {
    kStatusOk = 0,
    kStatusSingular = 1,
    kStatusNonfinite = 2,
    kStatusAborted = 3 // a bounded inter-block wait ran out (never expected)
};

struct PivotKey {
    double absval; // the rule's score (|value| for the paper's rule), -inf
                   // for "no candidate"; larger is better
    double value;  // the signed entry (the pivot keeps its sign)
    int colid;     // original column index (tie-break)
    int slot;      // where the entry sits in the current row
};

__device__ __forceinline__ PivotKey no_candidate()
{
    PivotKey k;
    k.absval = -INFINITY;
    k.value = 0.0;
    k.colid = INT_MAX;
    k.slot = -1;
    return k;
}

__device__ __forceinline__ bool better(const PivotKey& a, const PivotKey& b)
{
    return a.absval > b.absval || (a.absval == b.absval && a.colid < b.colid);
}

// Pivot-column rules.  The paper's rule is the largest |a| (Section 2.2);
// Section 1 describes two earlier ones that it argues against: the first
// non-zero entry of the row (Beliakov) and the non-zero entry whose |a| is
// closest to 1 (Haque).  Each is a score, larger is better, with ties to
// the smallest original column; the two earlier rules never take a zero.
enum : int { kRuleMaxAbs = 0, kRuleFirstNonzero = 1, kRuleClosestToOne = 2 };

// Offer one entry to a running key; returns false if the entry is not
// finite (the caller records that).
template <int RULE = kRuleMaxAbs>
__device__ __forceinline__ bool offer(PivotKey& k, double v, int colid,
                                      int slot)
{
    if (!isfinite(v)) return false;
    PivotKey c;
    if (RULE == kRuleMaxAbs) {
        c.absval = fabs(v);
    } else {
        if (v == 0.0) return true;
        c.absval = RULE == kRuleFirstNonzero ? 0.0 : -fabs(fabs(v) - 1.0);
    }
    c.value = v;
    c.colid = colid;
    c.slot = slot;
    if (better(c, k)) k = c;
    return true;
}

// Butterfly all-reduce over the 64 lanes of a wavefront.  `better` is a
// strict total order on distinct column ids, so every lane ends with the
// same winner.
__device__ __forceinline__ PivotKey wave_argmax(PivotKey k)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        PivotKey o;
        o.absval = __shfl_xor(k.absval, off, kWave);
        o.value = __shfl_xor(k.value, off, kWave);
        o.colid = __shfl_xor(k.colid, off, kWave);
        o.slot = __shfl_xor(k.slot, off, kWave);
        if (better(o, k)) k = o;
    }
    return k;
}

// Block-wide argmax and "any non-finite" for a block of NT threads.
// `sh` must hold NT/64 keys, `shflag` one int; both in LDS.
template <int NT>
__device__ __forceinline__ PivotKey block_argmax(PivotKey k, bool& bad,
                                                 PivotKey* sh, int* shflag)
{
    static_assert(NT % kWave == 0, "block must be whole wavefronts");
    if (threadIdx.x == 0) *shflag = 0;
    k = wave_argmax(k);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    if (lane == 0) sh[w] = k;
    if (bad) atomicOr(shflag, 1);
    __syncthreads();
    PivotKey r = sh[0];
#pragma unroll
    for (int i = 1; i < NT / kWave; ++i)
        if (better(sh[i], r)) r = sh[i];
    bad = *shflag != 0;
    __syncthreads();
    return r;
}

// Neumaier compensated summation (the log|pivot| accumulation of Figure 6,
// step 4.4, kept to ~1 ulp over thousands of terms).
struct Compensated {
    double sum;
    double comp;
};

__device__ __forceinline__ void comp_add(Compensated& a, double x)
{
    const double t = a.sum + x;
    if (fabs(a.sum) >= fabs(x))
        a.comp += (a.sum - t) + x;
    else
        a.comp += (x - t) + a.sum;
    a.sum = t;
}

__device__ __forceinline__ void comp_merge(Compensated& a, const Compensated& b)
{
    comp_add(a, b.sum);
    a.comp += b.comp;
}

// The XCD (accelerator complex) this wavefront runs on, 0..7 on a device
// that exposes all eight.
__device__ __forceinline__ int xcc_id()
{
    int x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 0xf;
}

// Operand loads through buffer descriptors: a lane whose element lies
// outside the operand takes an offset past the descriptor's range and reads
// 0 (the hardware's range check), so a load needs no branch, and nothing
// consumes its value before the LDS store that follows the K chunk's
// products (a load inside a branch, with its value used there, made the
// compiler wait for it at once).
constexpr uint32_t kOutOfRange = 0x7ffffff0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t operand_rsrc(const void* base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                             (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff),
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ T operand_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off);
template <>
__device__ __forceinline__ double operand_load<double>(__amdgpu_buffer_rsrc_t r,
                                                       uint32_t byte_off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
template <>
__device__ __forceinline__ float operand_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
} // namespace mc
