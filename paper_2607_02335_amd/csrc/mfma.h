// 16x16x4 matrix-core (MFMA) products in FP64 and FP32, and a wavefront
// barrier for LDS exchanges within one wavefront.
//
// Lane layout of one product D(16x16) += A(16x4) B(4x16) over a wavefront
// (lane l, group g = l / 16, column l % 16): lane l supplies A[l % 16][g]
// and B[g][l % 16] and holds four results D[row(l, r)][l % 16], r = 0..3.
#pragma once

#include <hip/hip_runtime.h>

namespace fem {

typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

template <typename C> struct Mfma;
template <> struct Mfma<double> {
    using V = v4d_t;
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // row of output register r held by lane l (column l % 16)
    __device__ static int row(int l, int r) { return 4 * r + l / 16; }
};
template <> struct Mfma<float> {
    using V = v4f_t;
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return 4 * (l / 16) + r; }
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace fem
