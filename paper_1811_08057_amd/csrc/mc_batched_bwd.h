// mc_batched_bwd.h -- arguments of the batched backward launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mc.h"
#include "mc_internal.h"

namespace mc {

struct BatchedBwdArgs {
    const void* const* LU_array;    // device array of device pointers (factors)
    const int64_t* n_array;         // device
    const int64_t* ld_array;        // device
    const int32_t* const* perm_array; // device array of device pointers
    int64_t batch;
    int64_t n_max;
    const double* grad_out;         // device, batch entries, or null (g = 1)
    const mc_result* fwd;           // device, batch entries, or null
    void* const* G_array;           // device array of device pointers (output)
    const int64_t* ldg_array;       // device
    int* counter;                   // [0] queue head, [1] item count
    int* items;                     // (matrix, column block) pairs
    void* inv;                      // per matrix: its diagonal blocks' inverses
    size_t inv_stride;              // bytes between two matrices' inverses
    size_t lds_elems;               // dynamic LDS of the launch, in elements
};

size_t batched_bwd_lds_bytes(int dtype, int64_t n_max);
size_t batched_bwd_workspace_bytes(int64_t batch, int64_t n_max, int dtype);
hipError_t launch_batched_backward(BatchedBwdArgs a, int dtype, void* work,
                                   hipStream_t stream);

} // namespace mc
