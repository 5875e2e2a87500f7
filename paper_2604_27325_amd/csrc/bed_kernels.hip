// bed_kernels.hip -- kernel entry points and their instantiations for gfx950.
#include "bed_internal.hpp"
#include "bed_syevd.hpp"

namespace bed {

// Waves per SIMD that two resident teams of a shape need (four SIMDs per CU);
// register allocation is capped accordingly.
template <int NMAX, int NT> struct Occ {
    static constexpr int teams_per_cu = NMAX >= 64 ? 2 : (NMAX >= 32 ? 4 : 8);
    static constexpr int v = (teams_per_cu * NT / 64 + 3) / 4;
    static constexpr int wpe = v < 1 ? 1 : (v > 8 ? 8 : v);
};
#define BED_OCC(NMAX, NT) __attribute__((amdgpu_waves_per_eu(Occ<NMAX, NT>::wpe)))

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT) BED_OCC(NMAX, NT)
k_syevd_uniform(const T *__restrict__ A, int n, int64_t batch, T *__restrict__ lam,
                T *__restrict__ Q, int32_t *__restrict__ info, int leaf)
{
    __shared__ Smem<T, NMAX, NT> S;
    const int64_t b = blockIdx.x;
    if (b >= batch) return;
    const int64_t n2 = (int64_t)n * n;
    syevd_team<T, NMAX, NT>(A + b * n2, n, lam + b * n, Q ? Q + b * n2 : nullptr,
                            info ? info + b : nullptr, S, threadIdx.x, leaf);
}

// Uniform batch of tridiagonal matrices: matrix b is the diagonal (n values)
// then the off-diagonal (n - 1 values) at tri + 2 n b.  Without Q, ends
// (nullable) receives the first and last rows of each eigenvector matrix at
// ends + 2 n b.
template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT) BED_OCC(NMAX, NT)
k_syevd_tri(const T *__restrict__ tri, int n, int64_t batch, T *__restrict__ lam,
            T *__restrict__ Q, int32_t *__restrict__ info, T *__restrict__ ends, int leaf)
{
    __shared__ Smem<T, NMAX, NT> S;
    const int64_t b = blockIdx.x;
    if (b >= batch) return;
    const int64_t n2 = (int64_t)n * n;
    syevd_team<T, NMAX, NT, true>(tri + b * 2 * n, n, lam + b * n, Q ? Q + b * n2 : nullptr,
                                  info ? info + b : nullptr, S, threadIdx.x, leaf,
                                  ends ? ends + b * 2 * n : nullptr);
}

// Static schedule: workgroup b solves item b.  The hardware dispatcher
// already hands a freed compute unit the next workgroup, so a finished team's
// slot is refilled at once.
template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT) BED_OCC(NMAX, NT)
k_syevd_list(const T *__restrict__ A, T *__restrict__ lam, T *__restrict__ Q,
             int32_t *__restrict__ info, const WorkItem *__restrict__ items, int count, int leaf)
{
    __shared__ Smem<T, NMAX, NT> S;
    if ((int)blockIdx.x >= count) return;
    const WorkItem w = items[blockIdx.x];
    syevd_team<T, NMAX, NT>(A + w.offA, w.n, lam + w.offL, Q ? Q + w.offA : nullptr,
                            info ? info + w.idx : nullptr, S, threadIdx.x, leaf);
}

// Persistent schedule: a fixed grid whose workgroups take matrices from a
// device counter until the list is exhausted, so the batch shrinks as work
// completes (Sec. 2.3.4, Eq. (22)).  The last workgroup to finish resets the
// counters, so the launch can be replayed from a graph without a memset.
template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT) BED_OCC(NMAX, NT)
k_syevd_persist(const T *__restrict__ A, T *__restrict__ lam, T *__restrict__ Q,
                int32_t *__restrict__ info, const WorkItem *__restrict__ items, int count,
                int *counter, int leaf)
{
    __shared__ Smem<T, NMAX, NT> S;
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(&counter[0], 1);
        __syncthreads();
        const int it = cur;
        __syncthreads();
        if (it >= count) break;
        const WorkItem w = items[it];
        // opaque thread index: per-thread addresses are formed anew for each
        // matrix instead of being held (and spilled) across the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        syevd_team<T, NMAX, NT>(A + w.offA, w.n, lam + w.offL, Q ? Q + w.offA : nullptr,
                                info ? info + w.idx : nullptr, S, tid, leaf);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counter[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&counter[0], 0);
            atomicExch(&counter[1], 0);
        }
    }
}

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT) BED_OCC(NMAX, NT)
k_syevd_ptrlist(const PtrItem *__restrict__ items, int count, int leaf)
{
    __shared__ Smem<T, NMAX, NT> S;
    if ((int)blockIdx.x >= count) return;
    const PtrItem w = items[blockIdx.x];
    syevd_team<T, NMAX, NT>((const T *)w.A, w.n, (T *)w.lam, (T *)w.Q, w.info, S, threadIdx.x,
                            leaf);
}

// ---------------------------------------------------------------- dispatch
#define BED_SHAPES(X) \
    X(16, 64) X(32, 64) X(32, 128) X(32, 256) X(64, 64) X(64, 128) X(64, 256) X(64, 512)

bool team_supported(bed_dtype dt, TeamShape ts)
{
    (void)dt;
    if (!leaf_supported(ts.leaf)) return false;
#define X(NM, NTT) if (ts.nmax == NM && ts.nt == NTT) return true;
    BED_SHAPES(X)
#undef X
    return false;
}

template <typename T>
static hipError_t uniform_t(TeamShape ts, const void *A, int n, int64_t batch, void *lam, void *Q,
                            int32_t *info, hipStream_t s)
{
#define X(NM, NTT)                                                                          \
    if (ts.nmax == NM && ts.nt == NTT) {                                                    \
        hipLaunchKernelGGL((k_syevd_uniform<T, NM, NTT>), dim3((unsigned)batch), dim3(NTT), \
                           0, s, (const T *)A, n, batch, (T *)lam, (T *)Q, info, ts.leaf);  \
        return hipGetLastError();                                                           \
    }
    BED_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_tri(TeamShape ts, const float *tri, int n, int64_t batch, float *lam, float *Q,
                      int32_t *info, float *ends, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    if (!leaf_supported(ts.leaf)) return hipErrorInvalidValue;
#define X(NM, NTT)                                                                          \
    if (ts.nmax == NM && ts.nt == NTT) {                                                    \
        hipLaunchKernelGGL((k_syevd_tri<float, NM, NTT>), dim3((unsigned)batch), dim3(NTT), \
                           0, s, tri, n, batch, lam, Q, info, ends, ts.leaf);               \
        return hipGetLastError();                                                           \
    }
    X(32, 128)
    X(32, 256)
    X(64, 512)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_uniform(bed_dtype dt, TeamShape ts, const void *A, int n, int64_t batch,
                          void *lam, void *Q, int32_t *info, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    return dt == BED_F32 ? uniform_t<float>(ts, A, n, batch, lam, Q, info, s)
                         : uniform_t<double>(ts, A, n, batch, lam, Q, info, s);
}

template <typename T>
static hipError_t list_t(TeamShape ts, const void *A, void *lam, void *Q, int32_t *info,
                         const WorkItem *items, int count, int *counter, int grid, hipStream_t s)
{
#define X(NM, NTT)                                                                             \
    if (ts.nmax == NM && ts.nt == NTT) {                                                       \
        if (counter)                                                                           \
            hipLaunchKernelGGL((k_syevd_persist<T, NM, NTT>), dim3((unsigned)grid), dim3(NTT), \
                               0, s, (const T *)A, (T *)lam, (T *)Q, info, items, count,       \
                               counter, ts.leaf);                                              \
        else                                                                                   \
            hipLaunchKernelGGL((k_syevd_list<T, NM, NTT>), dim3((unsigned)count), dim3(NTT),   \
                               0, s, (const T *)A, (T *)lam, (T *)Q, info, items, count,       \
                               ts.leaf);                                                       \
        return hipGetLastError();                                                              \
    }
    BED_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_list(bed_dtype dt, TeamShape ts, const void *A, void *lam, void *Q,
                       int32_t *info, const WorkItem *items, int count, int *counter, int grid,
                       hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dt == BED_F32 ? list_t<float>(ts, A, lam, Q, info, items, count, counter, grid, s)
                         : list_t<double>(ts, A, lam, Q, info, items, count, counter, grid, s);
}

template <typename T>
static hipError_t ptrlist_t(TeamShape ts, const PtrItem *items, int count, hipStream_t s)
{
#define X(NM, NTT)                                                                            \
    if (ts.nmax == NM && ts.nt == NTT) {                                                      \
        hipLaunchKernelGGL((k_syevd_ptrlist<T, NM, NTT>), dim3((unsigned)count), dim3(NTT), 0, \
                           s, items, count, ts.leaf);                                         \
        return hipGetLastError();                                                             \
    }
    BED_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_ptrlist(bed_dtype dt, TeamShape ts, const PtrItem *items, int count,
                          hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dt == BED_F32 ? ptrlist_t<float>(ts, items, count, s)
                         : ptrlist_t<double>(ts, items, count, s);
}

template <typename T>
static int bpc_t(TeamShape ts)
{
    int nb = 0;
#define X(NM, NTT)                                                                       \
    if (ts.nmax == NM && ts.nt == NTT) {                                                 \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_syevd_persist<T, NM, NTT>, \
                                                         NTT, 0) != hipSuccess)          \
            nb = 1;                                                                      \
        return nb > 0 ? nb : 1;                                                          \
    }
    BED_SHAPES(X)
#undef X
    return 1;
}

int blocks_per_cu(bed_dtype dt, TeamShape ts)
{
    return dt == BED_F32 ? bpc_t<float>(ts) : bpc_t<double>(ts);
}

}  // namespace bed
