// bed_device.hpp -- wave-level helpers for gfx950 (CDNA4, wave64).
//
// Cross-lane traffic inside a wave uses DPP (quad permutes, row mirrors) and
// the gfx950 permlane16/permlane32 swaps -- plain VALU operations, no LDS
// round trip.  Cross-wave traffic goes through LDS plus a workgroup barrier.
// A "team" is the set of threads that cooperate on one matrix: a whole
// workgroup (NT > 64) or a single wave (NT == 64).
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

// binary32: the hardware reciprocal (about 1 ulp) refined by one Newton step
// r' = r + r (1 - x r), and the hardware square root; binary64: IEEE division
// and square root.
__device__ __forceinline__ float f_rcp(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double f_rcp(double x) { return 1.0 / x; }
// Hardware reciprocal alone (about 1 ulp in FP32): for sums whose own
// rounding dominates, such as the secular function's terms.
__device__ __forceinline__ float f_rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double f_rcp_fast(double x) { return 1.0 / x; }
__device__ __forceinline__ float f_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// 1/sqrt(x): hardware estimate plus one Newton step (FP32); exact in FP64
__device__ __forceinline__ float f_rsqrt(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    return y * fmaf(-0.5f * x * y, y, 1.5f);
}
__device__ __forceinline__ double f_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ double f_sqrt(double x) { return sqrt(x); }
// binary64 hardware estimates refined by one Newton step, r' = r + r (1 - x r)
// and y' = y (3/2 - x y^2 / 2): the relative error squares, from the
// estimate's (at least 2^-22) to below 1e-12.  Used where binary64 arithmetic
// only has to keep its rounding far below binary32's unit roundoff.
__device__ __forceinline__ double d_rcp_nr(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double d_rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ float f_div(float a, float b) { return a * f_rcp(b); }
__device__ __forceinline__ double f_div(double a, double b) { return a / b; }

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

// Biased binary exponent field of x (0 for zero and subnormals) and the exact
// power of two 2^s (|s| at most SMAX, so that it stays a normal number).
__device__ __forceinline__ int exp_field(float x) { return (int)((__float_as_uint(x) >> 23) & 0xFFu); }
__device__ __forceinline__ int exp_field(double x)
{
    return (int)(((uint64_t)__double_as_longlong(x) >> 52) & 0x7FFu);
}
template <typename T> struct fexp;
template <> struct fexp<float> {
    static constexpr int BIAS = 127, SMAX = 100;
    static __device__ __forceinline__ float pow2(int s) { return __uint_as_float((uint32_t)(BIAS + s) << 23); }
};
template <> struct fexp<double> {
    static constexpr int BIAS = 1023, SMAX = 1000;
    static __device__ __forceinline__ double pow2(int s)
    {
        return __longlong_as_double((long long)((uint64_t)(BIAS + s) << 52));
    }
};

// ---- cross-lane moves --------------------------------------------------------
// DPP controls: quad_perm [1,0,3,2] = 0xB1 (lane ^ 1), [2,3,0,1] = 0x4E
// (lane ^ 2), row_half_mirror = 0x141 (lane ^ 7 within 8), row_mirror = 0x140
// (lane ^ 15 within 16).
template <int CTRL> __device__ __forceinline__ uint32_t dpp32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)x, CTRL, 0xF, 0xF, false);
}
// Value of lane ^ M within each quad (M = 1, 2, 3; quad_perm [3,2,1,0] = 0x1B
// is lane ^ 3).
template <int M> __device__ __forceinline__ uint32_t qxor32(uint32_t x)
{
    static_assert(M >= 0 && M <= 3, "quad lane mask");
    if constexpr (M == 0) return x;
    else if constexpr (M == 1) return dpp32<0xB1>(x);
    else if constexpr (M == 2) return dpp32<0x4E>(x);
    else return dpp32<0x1B>(x);
}
template <int M> __device__ __forceinline__ float qxor(float x)
{
    return __uint_as_float(qxor32<M>(__float_as_uint(x)));
}
template <int M> __device__ __forceinline__ int qxor(int x) { return (int)qxor32<M>((uint32_t)x); }
template <int M> __device__ __forceinline__ double qxor(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = qxor32<M>((uint32_t)b), hi = qxor32<M>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Value of lane ^ 16 (permlane16_swap exchanges odd rows of its first operand
// with even rows of its second) and of lane ^ 32 (permlane32_swap exchanges the
// upper half of its first operand with the lower half of its second).
__device__ __forceinline__ uint32_t xor16_32(uint32_t x, int lane)
{
    auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return ((lane >> 4) & 1) ? p[0] : p[1];
}
__device__ __forceinline__ uint32_t xor32_32(uint32_t x, int lane)
{
    auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane >= 32) ? p[0] : p[1];
}

// Generic "value held by lane ^ MASK-pattern" for float / double / int.
template <int STEP> __device__ __forceinline__ uint32_t xmove32(uint32_t x, int lane)
{
    if constexpr (STEP == 1) return dpp32<0xB1>(x);
    else if constexpr (STEP == 2) return dpp32<0x4E>(x);
    else if constexpr (STEP == 4) return dpp32<0x141>(x);
    else if constexpr (STEP == 8) return dpp32<0x140>(x);
    else if constexpr (STEP == 16) return xor16_32(x, lane);
    else return xor32_32(x, lane);
}
template <int STEP> __device__ __forceinline__ float xmove(float x, int lane)
{
    return __uint_as_float(xmove32<STEP>(__float_as_uint(x), lane));
}
template <int STEP> __device__ __forceinline__ int xmove(int x, int lane)
{
    return (int)xmove32<STEP>((uint32_t)x, lane);
}
template <int STEP> __device__ __forceinline__ double xmove(double x, int lane)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = xmove32<STEP>((uint32_t)b, lane);
    const uint32_t hi = xmove32<STEP>((uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum / product / max over aligned groups of W consecutive lanes (W a power of
// two).  The partner pattern is a butterfly (xor 1, 2, then mirrors inside
// 8/16 lanes, then row swaps), so every lane of a group gets a bit-identical
// result.
template <int W, typename T> __device__ __forceinline__ T group_sum(T x, int lane)
{
    if constexpr (W >= 2) x += xmove<1>(x, lane);
    if constexpr (W >= 4) x += xmove<2>(x, lane);
    if constexpr (W >= 8) x += xmove<4>(x, lane);
    if constexpr (W >= 16) x += xmove<8>(x, lane);
    if constexpr (W >= 32) x += xmove<16>(x, lane);
    if constexpr (W >= 64) x += xmove<32>(x, lane);
    return x;
}
template <int W, typename T> __device__ __forceinline__ T group_prod(T x, int lane)
{
    if constexpr (W >= 2) x *= xmove<1>(x, lane);
    if constexpr (W >= 4) x *= xmove<2>(x, lane);
    if constexpr (W >= 8) x *= xmove<4>(x, lane);
    if constexpr (W >= 16) x *= xmove<8>(x, lane);
    if constexpr (W >= 32) x *= xmove<16>(x, lane);
    if constexpr (W >= 64) x *= xmove<32>(x, lane);
    return x;
}
template <int W> __device__ __forceinline__ int group_min(int x, int lane)
{
    if constexpr (W >= 2) x = min(x, xmove<1>(x, lane));
    if constexpr (W >= 4) x = min(x, xmove<2>(x, lane));
    if constexpr (W >= 8) x = min(x, xmove<4>(x, lane));
    if constexpr (W >= 16) x = min(x, xmove<8>(x, lane));
    if constexpr (W >= 32) x = min(x, xmove<16>(x, lane));
    if constexpr (W >= 64) x = min(x, xmove<32>(x, lane));
    return x;
}
template <int W> __device__ __forceinline__ int group_max(int x, int lane)
{
    if constexpr (W >= 2) x = max(x, xmove<1>(x, lane));
    if constexpr (W >= 4) x = max(x, xmove<2>(x, lane));
    if constexpr (W >= 8) x = max(x, xmove<4>(x, lane));
    if constexpr (W >= 16) x = max(x, xmove<8>(x, lane));
    if constexpr (W >= 32) x = max(x, xmove<16>(x, lane));
    if constexpr (W >= 64) x = max(x, xmove<32>(x, lane));
    return x;
}
template <typename T> __device__ __forceinline__ T wave_sum(T x, int lane)
{
    return group_sum<64>(x, lane);
}

// Broadcast of one lane's value to the whole wave (lane index uniform).
__device__ __forceinline__ float bcast(float x, int src)
{
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(x), src));
}
__device__ __forceinline__ double bcast(double x, int src)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ int bcast(int x, int src) { return __builtin_amdgcn_readlane(x, src); }

// Inclusive prefix sum over the 64 lanes of a wave (row shifts, then the two
// row broadcasts), no LDS.
template <int CTRL, int ROWMASK> __device__ __forceinline__ uint32_t dppm32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0, (int)x, CTRL, ROWMASK, 0xF, true);
}
template <int CTRL, int ROWMASK> __device__ __forceinline__ float dppm(float x)
{
    return __uint_as_float(dppm32<CTRL, ROWMASK>(__float_as_uint(x)));
}
template <int CTRL, int ROWMASK> __device__ __forceinline__ double dppm(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = dppm32<CTRL, ROWMASK>((uint32_t)b);
    const uint32_t hi = dppm32<CTRL, ROWMASK>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <typename T> __device__ __forceinline__ T wave_prefix_sum(T x)
{
    x += dppm<0x111, 0xF>(x);  // row_shr:1 (out-of-row sources read 0)
    x += dppm<0x112, 0xF>(x);  // row_shr:2
    x += dppm<0x114, 0xF>(x);  // row_shr:4
    x += dppm<0x118, 0xF>(x);  // row_shr:8
    x += dppm<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dppm<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// Sum over the whole wave, returned as a wave-uniform value: row sums by four
// DPP butterflies, rows combined by the two row broadcasts into lane 63.
template <typename T> __device__ __forceinline__ T wave_total(T x)
{
    x += xmove<1>(x, 0);
    x += xmove<2>(x, 0);
    x += xmove<4>(x, 0);
    x += xmove<8>(x, 0);
    x += dppm<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dppm<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return bcast(x, 63);
}

// binary64 sum over the whole wave, in every lane.  A 64-bit DPP exchange
// takes two 32-bit moves, so the four butterfly stages inside rows of 16 use
// moves that read only valid lanes (no old value to clear), and the rows are
// combined by the two permlane swaps, whose two outputs together hold every
// row pair (a + b is the pair sum in every lane, so nothing is selected).
template <int CTRL> __device__ __forceinline__ double dpp_move64(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double wave_sum_all(double x)
{
    x += dpp_move64<0xB1>(x);   // lane ^ 1
    x += dpp_move64<0x4E>(x);   // lane ^ 2
    x += dpp_move64<0x141>(x);  // lane ^ 7 within 8
    x += dpp_move64<0x140>(x);  // lane ^ 15 within 16
    uint64_t b = (uint64_t)__double_as_longlong(x);
    auto l16 = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
    auto h16 = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    x = __longlong_as_double((long long)(((uint64_t)h16[0] << 32) | l16[0])) +
        __longlong_as_double((long long)(((uint64_t)h16[1] << 32) | l16[1]));
    b = (uint64_t)__double_as_longlong(x);
    auto l32 = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
    auto h32 = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)h32[0] << 32) | l32[0])) +
           __longlong_as_double((long long)(((uint64_t)h32[1] << 32) | l32[1]));
}
__device__ __forceinline__ float wave_sum_all(float x) { return wave_total(x); }

// Bits [lo, hi) of a 64-bit lane mask.
__device__ __forceinline__ uint64_t lane_range(int lo, int hi)
{
    uint64_t up = (hi >= 64) ? ~0ull : ((1ull << hi) - 1ull);
    uint64_t dn = (lo >= 64) ? ~0ull : ((1ull << lo) - 1ull);
    return up & ~dn;
}

}  // namespace bed
