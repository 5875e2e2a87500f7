// bed_gemm.hpp -- products of small square matrices held in LDS by one team,
// on 16x16x4 matrix-core tiles (bed_mfma.hpp), for the kernels that work on a
// finished eigendecomposition: the backward of the decomposition and the
// spectral matrix functions Q f(Lambda) Q^T with their backward.
//
// Matrices are NMAX x NMAX, row-major with leading dimension LDS_LD(NMAX) =
// NMAX + 2: a 16-lane row of an MFMA operand (16 rows, 2 k values per half
// wave) then falls on distinct banks when it walks down a column.  Only the
// leading n x n block is meaningful; the rest (up to 16-aligned n and to the
// 4-aligned k range) must hold zeros, so that every product of the padded
// blocks is exact and zero outside n x n.
#pragma once

#include "bed_device.hpp"
#include "bed_mfma.hpp"

namespace bed {

template <int NMAX> struct Lds {
    static constexpr int LD = NMAX + 2;
    static constexpr int SIZE = NMAX * LD;
};

// C = op(A) op(B) for the live 16x16 tiles of an n x n product; op(X) = X^T
// when the flag is set.  Wave w computes tiles w, w + NW, ...  Lane l supplies
// A[i0 + l%16][k] and B[k][j0 + l%16] for k = 4 s + l/16.  No team barrier.
template <typename T, int NMAX, int NT, bool TA, bool TB>
__device__ __forceinline__ void team_gemm(const T* __restrict__ A, const T* __restrict__ B,
                                          T* __restrict__ C, const int n, const int t)
{
    using MF = Mf<T>;
    constexpr int LD = Lds<NMAX>::LD;
    constexpr int RT = NMAX / 16;
    constexpr int NW = NT / 64;
    const int lane = t & 63, wave = t >> 6;
    const int i16 = lane & 15, kk = lane >> 4;
    const int nt = (n + 15) >> 4;
    const int ks = (n + 3) >> 2;
    for (int tile = wave; tile < RT * RT; tile += NW) {
        const int ti = tile % RT, tj = tile / RT;
        if (ti >= nt || tj >= nt) continue;
        const int i = 16 * ti + i16, j = 16 * tj + i16;
        typename MF::acc acc = MF::zero();
        for (int s = 0; s < ks; ++s) {
            const int k = 4 * s + kk;
            const T a = TA ? A[k * LD + i] : A[i * LD + k];
            const T b = TB ? B[j * LD + k] : B[k * LD + j];
            acc = MF::mma(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) C[(16 * ti + MF::crow(lane, v)) * LD + j] = acc[v];
    }
}

// Global n x n row-major matrix -> LDS NMAX x NMAX (zeros outside n x n);
// transpose = true stores G^T.  src == nullptr loads zeros.
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void team_load(const T* __restrict__ src, T* __restrict__ dst,
                                          const int n, const int t, const bool transpose = false)
{
    constexpr int LD = Lds<NMAX>::LD;
    for (int e = t; e < NMAX * NMAX; e += NT) {
        const int i = e / NMAX, j = e % NMAX;
        const bool in = i < n && j < n && src != nullptr;
        const T v = in ? src[i * n + j] : T(0);
        if (transpose) dst[j * LD + i] = v;
        else dst[i * LD + j] = v;
    }
}

// LDS n x n block -> global n x n row-major.
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void team_store(const T* __restrict__ src, T* __restrict__ dst,
                                           const int n, const int t)
{
    constexpr int LD = Lds<NMAX>::LD;
    for (int e = t; e < n * n; e += NT) {
        const int i = e / n, j = e - (e / n) * n;
        dst[e] = src[i * LD + j];
    }
}

}  // namespace bed
