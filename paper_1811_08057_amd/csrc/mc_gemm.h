// mc_gemm.h -- the trailing update of the blocked path on MFMA:
//     C[r0 + i][c0 + j] <- C[r0 + i][colsrc[c0 + j]] - sum_k L[i][k] U[k][c0 + j]
// for 0 <= i < M, 0 <= j < N, 0 <= k < K (K = panel width).  C is updated
// in place; colsrc maps each destination column to the position its old
// value sits at (the panel's column exchanges, see mc_blocked.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_internal.h"

namespace mc {

template <typename T>
struct GemmArgs {
    T* C;
    int64_t ldc;
    int64_t r0, c0; // first row / column of the updated block
    int64_t M, N;
    int K;
    const T* L; // M x K, row stride ldl (the rows' multipliers)
    int64_t ldl;
    const T* U; // K x (c0 + N), row stride ldu (the factored panel rows)
    int64_t ldu;
    const int* colsrc;
    const DevState* state;
    // Non-null: leave XCD 0 alone (for an update running beside a panel
    // chain there).  The blocks that land on XCD 0 leave before any memory
    // access; the others take tiles from *tile_ctr, which must be zero at
    // the launch, until none are left.
    unsigned int* tile_ctr = nullptr;
};

// update: MC_UPDATE_NATIVE (FP64 MFMA for double, FP32 MFMA for float),
// MC_UPDATE_F32 (float only), MC_UPDATE_BF16X3 (float only).
template <typename T>
hipError_t launch_trailing_update(const GemmArgs<T>& g, int update,
                                  hipStream_t stream);

} // namespace mc
