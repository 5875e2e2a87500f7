// bed_probe.hip -- instrumented build of the uniform-batch solver, for
// measurement only (separate library, never on the product path).  The same
// syevd_team code is compiled with its phase markers defined:
//   BED_PHASE(id)   thread 0 of each team stores the 100 MHz real-time clock
//                   (s_memrealtime) at phase boundary id into marks[b][id];
//   BED_DEFL(t1,t2) thread 0 adds the type-1 and type-2 deflations of each
//                   merge depth into defl[b][0], defl[b][1];
//   BED_HSTEP(k,id) lane 0 of wave 0 stores the shader clock (s_memtime) at
//                   sub-step id of the middle Householder step (k = NMAX/2)
//                   into steps[b][id]; after the last sub-step a second stamp
//                   follows at once, so that a marker's own cost is known.
// Reading the shader clock waits for outstanding scalar and LDS operations, so
// the step breakdown slightly lengthens the step it measures; the phase
// markers cost one store each.
#include <hip/hip_runtime.h>

#include "../../include/bed_probe.h"

namespace bed {
namespace probe {
__device__ long long *g_marks;
__device__ long long *g_steps;
__device__ long long *g_defl;
}  // namespace probe
}  // namespace bed

#define BED_PHASE(id)                                                                    \
    do {                                                                                 \
        if (threadIdx.x == 0)                                                            \
            ::bed::probe::g_marks[(long long)blockIdx.x * BED_PROBE_PHASES + (id)] =     \
                (long long)wall_clock64();                                               \
    } while (0)
#define BED_HSTEP(k, id)                                                                 \
    do {                                                                                 \
        if ((k) == NMAX / 2 && wave == 0 && lane == 0) {                                 \
            long long *st_ = ::bed::probe::g_steps + (long long)blockIdx.x * BED_PROBE_SUBSTEPS; \
            st_[(id)] = (long long)clock64();                                            \
            if ((id) == 8) st_[9] = (long long)clock64(); /* marker's own cost */        \
        }                                                                                \
    } while (0)

#define BED_DEFL(type1, type2)                                                         \
    do {                                                                                 \
        const int t1_ = (type1), t2_ = (type2);                                          \
        if (::bed::probe::g_defl && threadIdx.x == 0) {                                  \
            ::bed::probe::g_defl[2 * (long long)blockIdx.x] += t1_;                      \
            ::bed::probe::g_defl[2 * (long long)blockIdx.x + 1] += t2_;                  \
        }                                                                                \
    } while (0)

#include "bed_internal.hpp"
#include "bed_syevd.hpp"

namespace bed {

template <typename T, int NMAX, int NT>
__global__ void __launch_bounds__(NT)
k_probe_uniform(const T *__restrict__ A, int n, int64_t batch, T *__restrict__ lam,
                T *__restrict__ Q)
{
    __shared__ Smem<T, NMAX, NT> S;
    const int64_t b = blockIdx.x;
    if (b >= batch) return;
    const int64_t n2 = (int64_t)n * n;
    syevd_team<T, NMAX, NT>(A + b * n2, n, lam + b * n, Q ? Q + b * n2 : nullptr, nullptr, S,
                            threadIdx.x, leaf_default(NMAX));
}

#define BED_PROBE_SHAPES(X) X(16, 64) X(32, 64) X(32, 128) X(32, 256) X(64, 256) X(64, 512)

template <typename T>
static hipError_t probe_t(int nt, const void *A, int n, int64_t batch, void *lam, void *Q,
                          hipStream_t s)
{
    const int nmax = n <= 16 ? 16 : (n <= 32 ? 32 : 64);
#define X(NM, NTT)                                                                          \
    if (nmax == NM && nt == NTT) {                                                          \
        hipLaunchKernelGGL((k_probe_uniform<T, NM, NTT>), dim3((unsigned)batch), dim3(NTT), \
                           0, s, (const T *)A, n, batch, (T *)lam, (T *)Q);                 \
        return hipGetLastError();                                                           \
    }
    BED_PROBE_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace bed

extern "C" int32_t bed_probe_phases(int32_t dtype, int32_t threads, int32_t n, int64_t batch,
                                    const void *A, void *lambda, void *Q, long long *marks,
                                    long long *steps, long long *defl, void *stream)
{
    if (n < 1 || n > 64 || batch < 1 || !A || !lambda || !marks || !steps) return 1;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(marks, 0, sizeof(long long) * batch * BED_PROBE_PHASES, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(steps, 0, sizeof(long long) * batch * BED_PROBE_SUBSTEPS, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(bed::probe::g_marks), &marks, sizeof(marks), 0,
                                   hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(bed::probe::g_steps), &steps, sizeof(steps), 0,
                                   hipMemcpyHostToDevice, s);
    if (e == hipSuccess && defl)
        e = hipMemsetAsync(defl, 0, sizeof(long long) * 2 * batch, s);
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(bed::probe::g_defl), &defl, sizeof(defl), 0,
                                   hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host values above are locals
    if (e == hipSuccess)
        e = dtype == 0 ? bed::probe_t<float>(threads, A, n, batch, lambda, Q, s)
                       : bed::probe_t<double>(threads, A, n, batch, lambda, Q, s);
    return e == hipSuccess ? 0 : 3;
}
