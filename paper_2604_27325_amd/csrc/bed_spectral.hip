// bed_spectral.hip -- spectral matrix functions on a finished decomposition
// A = Q diag(lambda) Q^T, for the differentiable meta-layer use that motivates
// the note (Sec. 1; matrix square root and whitening among them):
//
//   F = Q f(Lambda) Q^T,
//   dA = Q ( K o (Q^T sym(dF) Q) ) Q^T,  K_ij = (f(l_i) - f(l_j)) / (l_i - l_j),
//                                        K_ii = f'(l_i)
//
// (the first-order perturbation of f(A), Daleckii-Krein).  The divided
// differences are written without cancellation for every f.  One team per
// matrix; the products run on 16x16x4 matrix-core tiles out of LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bed_gemm.hpp"
#include "bed_host.hpp"
#include "bed_internal.hpp"

namespace bed {

__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double m_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float m_pow(float x, float p) { return powf(x, p); }
__device__ __forceinline__ double m_pow(double x, double p) { return pow(x, p); }

template <typename T>
__device__ __forceinline__ T fn_value(const int fn, const T x, const T p)
{
    switch (fn) {
    case BED_FN_SQRT: return m_sqrt(x);
    case BED_FN_INVSQRT: return T(1) / m_sqrt(x);
    case BED_FN_EXP: return m_exp(x);
    case BED_FN_LOG: return m_log(x);
    default: return m_pow(x, p);
    }
}

template <typename T>
__device__ __forceinline__ T fn_deriv(const int fn, const T x, const T p)
{
    switch (fn) {
    case BED_FN_SQRT: return T(0.5) / m_sqrt(x);
    case BED_FN_INVSQRT: return T(-0.5) / (x * m_sqrt(x));
    case BED_FN_EXP: return m_exp(x);
    case BED_FN_LOG: return T(1) / x;
    default: return p * m_pow(x, p - T(1));
    }
}

// (f(a) - f(b)) / (a - b), and f'(a) when a == b:
//   sqrt     1 / (sqrt a + sqrt b)
//   invsqrt  -1 / (sqrt a sqrt b (sqrt a + sqrt b))
//   exp      e^b expm1(a - b) / (a - b)
//   log      log1p((a - b) / b) / (a - b)
//   pow      b^p expm1(p log1p((a - b) / b)) / (a - b)
template <typename T>
__device__ __forceinline__ T fn_divdiff(const int fn, const T a, const T b, const T p)
{
    const T d = a - b;
    if (d == T(0)) return fn_deriv(fn, a, p);
    switch (fn) {
    case BED_FN_SQRT: return T(1) / (m_sqrt(a) + m_sqrt(b));
    case BED_FN_INVSQRT: {
        const T sa = m_sqrt(a), sb = m_sqrt(b);
        return T(-1) / (sa * sb * (sa + sb));
    }
    case BED_FN_EXP: return m_exp(b) * m_expm1(d) / d;
    case BED_FN_LOG: return m_log1p(d / b) / d;
    default: return m_pow(b, p) * m_expm1(p * m_log1p(d / b)) / d;
    }
}

template <typename T, int NMAX>
struct SpecSmem {
    static constexpr int SZ = Lds<NMAX>::SIZE;
    T Q[SZ];
    T X[SZ];
    T Y[SZ];
    T lam[NMAX], fl[NMAX];
};

// F = (Q diag(f(lambda))) Q^T
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void apply_team(const T *__restrict__ lam, const T *__restrict__ Q,
                                           T *__restrict__ F, const int n, const int fn,
                                           const T p, SpecSmem<T, NMAX> &S, const int t)
{
    constexpr int LD = Lds<NMAX>::LD;
    team_load<T, NMAX, NT>(Q, S.Q, n, t);
    for (int e = t; e < NMAX; e += NT) S.fl[e] = e < n ? fn_value(fn, lam[e], p) : T(0);
    __syncthreads();
    for (int e = t; e < NMAX * NMAX; e += NT) {
        const int i = e / NMAX, j = e % NMAX;
        S.Y[i * LD + j] = S.Q[i * LD + j] * S.fl[j];
    }
    __syncthreads();
    team_gemm<T, NMAX, NT, false, true>(S.Y, S.Q, S.X, n, t);
    __syncthreads();
    team_store<T, NMAX, NT>(S.X, F, n, t);
}

// dA = Q (K o sym(Q^T dF Q)) Q^T
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void spec_bwd_team(const T *__restrict__ lam, const T *__restrict__ Q,
                                              const T *__restrict__ dF, T *__restrict__ dA,
                                              const int n, const int fn, const T p,
                                              SpecSmem<T, NMAX> &S, const int t)
{
    constexpr int LD = Lds<NMAX>::LD;
    team_load<T, NMAX, NT>(Q, S.Q, n, t);
    team_load<T, NMAX, NT>(dF, S.X, n, t);
    for (int e = t; e < NMAX; e += NT) S.lam[e] = e < n ? lam[e] : T(0);
    __syncthreads();
    team_gemm<T, NMAX, NT, false, false>(S.X, S.Q, S.Y, n, t);  // Y = dF Q
    __syncthreads();
    team_gemm<T, NMAX, NT, true, false>(S.Q, S.Y, S.X, n, t);   // X = Q^T dF Q
    __syncthreads();
    for (int e = t; e < NMAX * NMAX; e += NT) {
        const int i = e / NMAX, j = e % NMAX;
        T v = T(0);
        if (i < n && j < n)
            v = fn_divdiff(fn, S.lam[i], S.lam[j], p) * T(0.5) * (S.X[i * LD + j] + S.X[j * LD + i]);
        S.Y[i * LD + j] = v;
    }
    __syncthreads();
    team_gemm<T, NMAX, NT, false, false>(S.Q, S.Y, S.X, n, t);  // X = Q S
    __syncthreads();
    team_gemm<T, NMAX, NT, false, true>(S.X, S.Q, S.Y, n, t);   // Y = X Q^T
    __syncthreads();
    team_store<T, NMAX, NT>(S.Y, dA, n, t);
}

// Uniform batch: offsets from the block index; list: one work item per block.
template <typename T, int NMAX, int NT, bool BWD>
__global__ void __launch_bounds__(NT)
k_spectral(const T *lam, const T *Q, const T *in, T *out, int n, int64_t batch,
           const WorkItem *items, int fn, T p)
{
    __shared__ SpecSmem<T, NMAX> S;
    int64_t offA, offL;
    int nn;
    if (items) {
        const WorkItem w = items[blockIdx.x];
        offA = w.offA;
        offL = w.offL;
        nn = w.n;
    } else {
        if ((int64_t)blockIdx.x >= batch) return;
        offA = (int64_t)blockIdx.x * n * n;
        offL = (int64_t)blockIdx.x * n;
        nn = n;
    }
    if constexpr (BWD)
        spec_bwd_team<T, NMAX, NT>(lam + offL, Q + offA, in + offA, out + offA, nn, fn, p, S,
                                   threadIdx.x);
    else
        apply_team<T, NMAX, NT>(lam + offL, Q + offA, out + offA, nn, fn, p, S, threadIdx.x);
}

template <typename T, bool BWD>
static hipError_t spectral_t(int nmax, const void *lam, const void *Q, const void *in, void *out,
                             int n, int64_t count, const WorkItem *items, int fn, double p,
                             hipStream_t s)
{
#define SPEC(NM, NTT)                                                                        \
    hipLaunchKernelGGL((k_spectral<T, NM, NTT, BWD>), dim3((unsigned)count), dim3(NTT), 0, s, \
                       (const T *)lam, (const T *)Q, (const T *)in, (T *)out, n, count, items, \
                       fn, (T)p)
    if (nmax <= 16) SPEC(16, 64);
    else if (nmax <= 32) SPEC(32, 256);
    else SPEC(64, 256);
#undef SPEC
    return hipGetLastError();
}

static hipError_t spectral_launch(bed_dtype dt, bool bwd, int nmax, const void *lam, const void *Q,
                                  const void *in, void *out, int n, int64_t count,
                                  const WorkItem *items, int fn, double p, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (dt == BED_F32)
        return bwd ? spectral_t<float, true>(nmax, lam, Q, in, out, n, count, items, fn, p, s)
                   : spectral_t<float, false>(nmax, lam, Q, in, out, n, count, items, fn, p, s);
    return bwd ? spectral_t<double, true>(nmax, lam, Q, in, out, n, count, items, fn, p, s)
               : spectral_t<double, false>(nmax, lam, Q, in, out, n, count, items, fn, p, s);
}

static bed_status spectral(bed_dtype dt, bool bwd, int64_t batch, const int32_t *n,
                           const void *lam, const void *Q, int32_t fn, double param,
                           const void *in, void *out, void *stream)
{
    bed_status st = check_sizes(dt, batch, n);
    if (st != BED_OK) return st;
    if (fn < BED_FN_SQRT || fn > BED_FN_POW) return fail(BED_ERR_INVALID_ARG, "unknown function %d", fn);
    if (batch == 0) return BED_OK;
    if ((st = check_ptr(lam, dt, "lambda", false)) != BED_OK) return st;
    if ((st = check_ptr(Q, dt, "Q", false)) != BED_OK) return st;
    if (bwd && (st = check_ptr(in, dt, "dF", false)) != BED_OK) return st;
    if ((st = check_ptr(out, dt, bwd ? "dA" : "F", false)) != BED_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool uniform = std::all_of(n, n + batch, [&](int32_t v) { return v == n[0]; });
    if (uniform) {
        hipError_t e = spectral_launch(dt, bwd, n[0], lam, Q, in, out, n[0], batch, nullptr, fn,
                                       param, s);
        return e == hipSuccess ? BED_OK : hip_fail(e, "spectral launch");
    }
    return with_worklist(dt, batch, n, s, [&](const WorkItem *items, int count, int nmax) {
        return spectral_launch(dt, bwd, nmax, lam, Q, in, out, 0, count, items, fn, param, s);
    });
}

}  // namespace bed

extern "C" bed_status bed_spectral_apply(bed_dtype dt, int64_t batch, const int32_t *n,
                                         const void *lambda, const void *Q, int32_t fn,
                                         double param, void *F, void *stream)
{
    return bed::spectral(dt, false, batch, n, lambda, Q, fn, param, nullptr, F, stream);
}

extern "C" bed_status bed_spectral_backward(bed_dtype dt, int64_t batch, const int32_t *n,
                                            const void *lambda, const void *Q, int32_t fn,
                                            double param, const void *dF, void *dA, void *stream)
{
    return bed::spectral(dt, true, batch, n, lambda, Q, fn, param, dF, dA, stream);
}
