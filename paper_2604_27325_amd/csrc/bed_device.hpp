// bed_device.hpp -- wave-level helpers for gfx950 (CDNA4, wave64).
//
// All cross-lane traffic inside a wave goes through ds_bpermute/DPP (via the
// HIP shuffle intrinsics); cross-wave traffic goes through LDS plus a
// workgroup barrier.  A "team" is the set of threads that cooperate on one
// matrix: a whole workgroup (NT > 64) or a single wave (NT == 64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bed {

template <typename T> struct fp;
template <> struct fp<float> {
    static constexpr float u = 0x1p-24f;  // unit roundoff of binary32
};
template <> struct fp<double> {
    static constexpr double u = 0x1p-53;  // unit roundoff of binary64
};

__device__ __forceinline__ float f_abs(float x) { return fabsf(x); }
__device__ __forceinline__ double f_abs(double x) { return fabs(x); }
__device__ __forceinline__ float f_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double f_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float f_hypot(float x, float y) { return hypotf(x, y); }
__device__ __forceinline__ double f_hypot(double x, double y) { return hypot(x, y); }
__device__ __forceinline__ float f_max(float x, float y) { return fmaxf(x, y); }
__device__ __forceinline__ double f_max(double x, double y) { return fmax(x, y); }
__device__ __forceinline__ float f_copysign(float x, float y) { return copysignf(x, y); }
__device__ __forceinline__ double f_copysign(double x, double y) { return copysign(x, y); }
__device__ __forceinline__ bool f_finite(float x) { return isfinite(x); }
__device__ __forceinline__ bool f_finite(double x) { return isfinite(x); }
template <typename T> __device__ __forceinline__ T f_nan();
template <> __device__ __forceinline__ float f_nan<float>() { return __builtin_nanf(""); }
template <> __device__ __forceinline__ double f_nan<double>() { return __builtin_nan(""); }

// Orders LDS traffic between the lanes of one wave: a wave executes its LDS
// instructions in order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NT>
__device__ __forceinline__ void team_sync()
{
    if constexpr (NT > 64)
        __syncthreads();
    else
        wave_sync();
}

template <typename T> __device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Sum / product over aligned groups of W consecutive lanes (W a power of two
// dividing 64).  Butterfly order makes every lane of a group bit-identical.
template <int W, typename T> __device__ __forceinline__ T group_sum(T x)
{
#pragma unroll
    for (int o = W / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
template <int W, typename T> __device__ __forceinline__ T group_prod(T x)
{
#pragma unroll
    for (int o = W / 2; o >= 1; o >>= 1) x *= __shfl_xor(x, o);
    return x;
}

// Bits [lo, hi) of a 64-bit lane mask.
__device__ __forceinline__ uint64_t lane_range(int lo, int hi)
{
    uint64_t up = (hi >= 64) ? ~0ull : ((1ull << hi) - 1ull);
    uint64_t dn = (lo >= 64) ? ~0ull : ((1ull << lo) - 1ull);
    return up & ~dn;
}

// Segmented inclusive scan over contiguous lane segments [lo, hi); returns
// the segment total to every lane of the segment.  Every lane of the wave
// must call it (lanes outside any segment pass lo = hi = lane, x = 0).
template <typename T> __device__ __forceinline__ T seg_sum(T x, int e, int lo, int hi)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (e - o >= lo) x += y;
    }
    return __shfl(x, hi > lo ? hi - 1 : e);
}
template <typename T> __device__ __forceinline__ T seg_max(T x, int e, int lo, int hi)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (e - o >= lo) x = f_max(x, y);
    }
    return __shfl(x, hi > lo ? hi - 1 : e);
}

}  // namespace bed
