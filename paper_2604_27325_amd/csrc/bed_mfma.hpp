// bed_mfma.hpp -- 16x16x4 matrix-core tiles (gfx950) for the dense products
// of the solver: the back-multiplication of each merge (Eq. (4)) and the
// Householder back-transform in compact-WY form.
//
// One MFMA step multiplies a 16x4 slice of A by a 4x16 slice of B into a
// 16x16 accumulator.  Lane l supplies A[l%16][kk] and B[kk][l%16] for the
// step's "hardware" k index kk = l/16.  The accumulator holds element v of
// lane l at row crow(l, v), column l%16:
//   binary32 (v_mfma_f32_16x16x4f32):  crow = 4*(l/16) + v
//   binary64 (v_mfma_f64_16x16x4f64):  crow = l/16 + 4*v
// Because crow(l, s) depends only on (l/16, s), an accumulator can feed the
// next product directly as its B operand: in step s every lane supplies its
// element s and the A operand uses the same row map crow(l, s).
#pragma once

#include "bed_device.hpp"

namespace bed {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mf;
template <> struct Mf<float> {
    using acc = f32x4;
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int crow(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mf<double> {
    using acc = f64x4;
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int crow(int lane, int v) { return (lane >> 4) + 4 * v; }
};

}  // namespace bed
