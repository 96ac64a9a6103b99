// mc_gmm.h -- arguments of the mixture log-likelihood launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mc.h"
#include "mc_internal.h"

namespace mc {

struct GmmArgs {
    const void* X;      // m x d points, row stride ldx
    int64_t m, d, ldx;
    const void* means;  // k x d, row stride ldmu
    int64_t ldmu, k;
    const double* log_weights;        // k
    const void* const* LU_array;      // k factor pointers (device array)
    const int64_t* ld_array;          // k
    const int32_t* const* perm_array; // k
    const mc_result* fwd;             // k factor results
    double* loglik;                   // m (output)
    double* total;                    // 1 (output) or null
    // workspace
    int* counter;
    double* Q;       // k x m Mahalanobis terms
    double* partial; // per-block sums of loglik
    void* slots;     // per workgroup: 64 right-hand sides of ldy elements
    int64_t ldy;
    void* inv;       // per component: its diagonal blocks' inverses
    size_t inv_stride;
};

int64_t gmm_ldy(int64_t d);
size_t gmm_workspace_bytes(int64_t m, int64_t d, int64_t k, int dtype);
hipError_t launch_gmm(GmmArgs a, int dtype, void* work, size_t work_bytes,
                      hipStream_t stream);

} // namespace mc
