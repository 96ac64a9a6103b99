// mc_mfma.h -- matrix-core (MFMA) operand policies for gfx950.
//
// Accumulator layouts (measured on gfx950 with one-hot operands):
//   v_mfma_f64_16x16x4f64:    D(i, j) in lane j + 16 (i mod 4), register i / 4
//   v_mfma_f32_16x16x4f32:    D(i, j) in lane j + 16 (i / 4),   register i mod 4
//   v_mfma_f32_16x16x32_bf16: as the f32 one.
// Operands: A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k (K = 4); in
// the bf16 form each lane holds k = 8 (lane / 16) + e, e = 0..7.
#pragma once

#include <hip/hip_runtime.h>

namespace mc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct MfmaF64 {
    using T = double;
    using Acc = d4;
    // row of accumulator register r held by `lane` (column = lane mod 16)
    __device__ static int drow(int lane, int r) { return (lane >> 4) + 4 * r; }
    __device__ static Acc mma(double a, double b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

struct MfmaF32 {
    using T = float;
    using Acc = f4;
    __device__ static int drow(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static Acc mma(float a, float b, Acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename T>
struct MfmaFor;
template <>
struct MfmaFor<double> {
    using P = MfmaF64;
};
template <>
struct MfmaFor<float> {
    using P = MfmaF32;
};

} // namespace mc
