// bed_backward.hip -- backward of the eigendecomposition A = Q diag(lam) Q^T:
//
//   dA = Q ( diag(dlam) + sym(F o (Q^T dQ)) ) Q^T,   sym(X) = (X + X^T)/2,
//   F_ij = 1/(lam_j - lam_i) (i != j), zero when |lam_i - lam_j| is within the
//   degeneracy guard.
//
// The note motivates the solver as a differentiable meta-layer (Sec. 1); the
// formula is the standard one for symmetric eigendecomposition.  One workgroup
// per matrix; the three products run on 16x16x4 matrix-core tiles out of LDS
// (bed_gemm.hpp).
#include "bed_device.hpp"
#include "bed_gemm.hpp"
#include "bed_internal.hpp"

namespace bed {

template <typename T, int NMAX>
struct BwdSmem {
    static constexpr int SZ = Lds<NMAX>::SIZE;
    T Q[SZ];
    T X[SZ];  // dQ, then S, then dA
    T Y[SZ];  // Q^T dQ, then Q S
    T lam[NMAX], dlam[NMAX];
    T lmax;
};

// One team per matrix: three n x n products on MFMA tiles out of LDS, with
// the guarded F applied between the first two.
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void bwd_team(const T *__restrict__ lam, const T *__restrict__ Q,
                                         const T *__restrict__ dlam, const T *__restrict__ dQ,
                                         T *__restrict__ dA, const int n, const T eps,
                                         BwdSmem<T, NMAX> &S, const int t)
{
    constexpr int LD = Lds<NMAX>::LD;
    team_load<T, NMAX, NT>(Q, S.Q, n, t);
    team_load<T, NMAX, NT>(dQ, S.X, n, t);
    for (int e = t; e < NMAX; e += NT) {
        S.lam[e] = e < n ? lam[e] : T(0);
        S.dlam[e] = (e < n && dlam) ? dlam[e] : T(0);
    }
    __syncthreads();
    if (t < 64) {
        T m = T(0);
        for (int e = t; e < n; e += 64) m = f_max(m, f_abs(S.lam[e]));
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = f_max(m, __shfl_xor(m, o));
        if (t == 0) S.lmax = m;
    }
    // Y = Q^T dQ
    team_gemm<T, NMAX, NT, true, false>(S.Q, S.X, S.Y, n, t);
    __syncthreads();
    // X = diag(dlam) + sym(F o Y), F_ij = 1/(lam_j - lam_i) outside the guard
    const T guard = eps * f_max(T(1), S.lmax);
    for (int e = t; e < NMAX * NMAX; e += NT) {
        const int i = e / NMAX, j = e % NMAX;
        T v = T(0);
        if (i < n && j < n) {
            if (i == j) {
                v = S.dlam[i];
            } else {
                const T gap = S.lam[j] - S.lam[i];
                v = f_abs(gap) > guard ? T(0.5) * f_div(S.Y[i * LD + j] - S.Y[j * LD + i], gap)
                                       : T(0);
            }
        }
        S.X[i * LD + j] = v;
    }
    __syncthreads();
    // Y = Q X, then X = Y Q^T = dA
    team_gemm<T, NMAX, NT, false, false>(S.Q, S.X, S.Y, n, t);
    __syncthreads();
    team_gemm<T, NMAX, NT, false, true>(S.Y, S.Q, S.X, n, t);
    __syncthreads();
    team_store<T, NMAX, NT>(S.X, dA, n, t);
}

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT)
k_bwd_list(const T *lam, const T *Q, const T *dlam, const T *dQ, T *dA, const WorkItem *items,
           int count, T eps)
{
    __shared__ BwdSmem<T, NMAX> S;
    for (int it = blockIdx.x; it < count; it += gridDim.x) {
        const WorkItem w = items[it];
        bwd_team<T, NMAX, NT>(lam + w.offL, Q + w.offA, dlam ? dlam + w.offL : nullptr,
                              dQ ? dQ + w.offA : nullptr, dA + w.offA, w.n, eps, S, threadIdx.x);
        __syncthreads();
    }
}

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT)
k_bwd_uniform(const T *lam, const T *Q, const T *dlam, const T *dQ, T *dA, int n, int64_t batch,
              T eps)
{
    __shared__ BwdSmem<T, NMAX> S;
    const int64_t b = blockIdx.x;
    if (b >= batch) return;
    const int64_t n2 = (int64_t)n * n;
    bwd_team<T, NMAX, NT>(lam + b * n, Q + b * n2, dlam ? dlam + b * n : nullptr,
                          dQ ? dQ + b * n2 : nullptr, dA + b * n2, n, eps, S, threadIdx.x);
}

template <typename T>
static hipError_t bwd_list_t(int nmax, const void *lam, const void *Q, const void *dlam,
                             const void *dQ, void *dA, const WorkItem *items, int count, double eps,
                             hipStream_t s)
{
#define BWD_L(NM, NTT)                                                                         \
    hipLaunchKernelGGL((k_bwd_list<T, NM, NTT>), dim3((unsigned)count), dim3(NTT), 0, s,       \
                       (const T *)lam, (const T *)Q, (const T *)dlam, (const T *)dQ, (T *)dA, \
                       items, count, (T)eps)
    if (nmax <= 16) BWD_L(16, 64);
    else if (nmax <= 32) BWD_L(32, 256);
    else BWD_L(64, 256);
#undef BWD_L
    return hipGetLastError();
}

template <typename T>
static hipError_t bwd_uniform_t(int nmax, const void *lam, const void *Q, const void *dlam,
                                const void *dQ, void *dA, int n, int64_t batch, double eps,
                                hipStream_t s)
{
#define BWD_U(NM, NTT)                                                                         \
    hipLaunchKernelGGL((k_bwd_uniform<T, NM, NTT>), dim3((unsigned)batch), dim3(NTT), 0, s,    \
                       (const T *)lam, (const T *)Q, (const T *)dlam, (const T *)dQ, (T *)dA, \
                       n, batch, (T)eps)
    if (nmax <= 16) BWD_U(16, 64);
    else if (nmax <= 32) BWD_U(32, 256);
    else BWD_U(64, 256);
#undef BWD_U
    return hipGetLastError();
}

hipError_t launch_backward(bed_dtype dt, int nmax, const void *lam, const void *Q,
                           const void *dlam, const void *dQ, void *dA, const WorkItem *items,
                           int count, double eps, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dt == BED_F32 ? bwd_list_t<float>(nmax, lam, Q, dlam, dQ, dA, items, count, eps, s)
                         : bwd_list_t<double>(nmax, lam, Q, dlam, dQ, dA, items, count, eps, s);
}

hipError_t launch_backward_uniform(bed_dtype dt, int nmax, const void *lam, const void *Q,
                                   const void *dlam, const void *dQ, void *dA, int n,
                                   int64_t batch, double eps, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    return dt == BED_F32
               ? bwd_uniform_t<float>(nmax, lam, Q, dlam, dQ, dA, n, batch, eps, s)
               : bwd_uniform_t<double>(nmax, lam, Q, dlam, dQ, dA, n, batch, eps, s);
}

}  // namespace bed
