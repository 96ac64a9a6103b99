// mc_batched.h -- the batched path's arguments and tuning table.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mc.h"
#include "mc_internal.h"

namespace mc {

// Size buckets of the tuning table: n <= 64, 128, 256, 512, 1024, larger.
constexpr int kTuneBuckets = 6;

__host__ __device__ inline int64_t tune_bucket_max(int k)
{
    return k >= kTuneBuckets - 1 ? INT64_MAX : ((int64_t)64 << k);
}

struct TuneTable {
    int64_t b[kTuneBuckets]; // panel width per bucket
    int tile[kTuneBuckets];  // trailing-update tile edge (32 or 64)
};

struct BatchArgs {
    const void* const* A_array; // device array of device pointers
    const int64_t* n_array;     // device
    const int64_t* lda_array;   // device
    int64_t batch;
    int64_t n_max;
    int update;
    TuneTable table;
    unsigned char* regions; // batch regions of region_stride bytes
    size_t region_stride;
    int* counter; // queue head
    int* order;   // matrices by decreasing size
    mc_result* out;
    // the factor call: device array of each matrix's perm output (the
    // matrices in A_array are then factored in place); null otherwise
    int32_t* const* perm_array = nullptr;
    // workgroups that land on XCD 0 leave at once (a blocked-path call may
    // run beside the launch, its column-split panels on XCD 0)
    int skip_xcc0 = 0;
};

// Process-wide: batched launches leave XCD 0 alone (read once per call).
int batched_spare_xcc0(int on);
bool batched_spare_xcc0_on();

size_t batched_region_bytes(int64_t n_max, int dtype, const TuneTable& t,
                            bool with_w = true);
size_t batched_lds_bytes(int dtype, const TuneTable& t);
hipError_t launch_batched(const BatchArgs& a, int dtype, size_t lds_bytes,
                          hipStream_t stream);

} // namespace mc
