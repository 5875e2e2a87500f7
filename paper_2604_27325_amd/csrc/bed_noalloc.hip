// bed_noalloc.hip -- bed_syevd_noalloc: the one-shot solve of bed_syevd with no
// allocation of any kind, for callers that cannot allocate device memory.
//
// A mixed-size batch needs a device work list (offsets and size of every
// matrix, grouped by size class).  Here it lives in `scratch`, a file-scope
// device array of fixed size that each GPU holds for the life of the process.
// The matrix sizes reach the device as kernel arguments (one byte per matrix,
// in chunks), so no host buffer has to outlive the call and no copy or memset
// is issued: one small kernel per chunk writes the chunk's work items, then
// one solver launch per size class reads them.  Matrices of a class run in
// input order.  Every call on a GPU rewrites that GPU's array, so two calls
// that overlap in time on one GPU race (documented in bed.h).
#include <hip/hip_runtime.h>

#include <mutex>

#include "bed_host.hpp"
#include "bed_internal.hpp"

namespace bed {

constexpr int NOALLOC_MAX = BED_NOALLOC_MAX_BATCH;
constexpr int CHUNK = 2048;       // matrices per list-building launch
constexpr int LIST_THREADS = 1024;

// The work list of the largest admissible batch: NOALLOC_MAX items of 24 bytes.
static __device__ __align__(256) unsigned char scratch[sizeof(WorkItem) * NOALLOC_MAX];

struct ChunkArgs {
    int64_t offA0, offL0;     // packed offsets of the chunk's first matrix
    int32_t b0, count;        // first batch index, matrices in the chunk
    int32_t cls_base[3];      // item index of the chunk's first matrix of each class
    uint8_t n[CHUNK];         // sizes (1..64)
};

// Exclusive scan over the block of one 64-bit value per thread.
__device__ __forceinline__ int64_t block_scan_excl(int64_t v, int64_t *sh, int64_t &total)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (t < 64) {
        int64_t w = (t < LIST_THREADS / 64) ? sh[t] : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(w, o);
            if (lane >= o) w += y;
        }
        if (t < LIST_THREADS / 64) sh[t] = w;  // inclusive sums of the waves
    }
    __syncthreads();
    const int64_t before = (wave > 0 ? sh[wave - 1] : 0) + x - v;
    total = sh[LIST_THREADS / 64 - 1];
    __syncthreads();
    return before;
}

__device__ __forceinline__ int class_of(int n) { return n <= 16 ? 0 : (n <= 32 ? 1 : 2); }

// Thread t handles matrices 2t and 2t + 1 of the chunk.
__global__ void __launch_bounds__(LIST_THREADS) k_noalloc_list(ChunkArgs a, WorkItem *items)
{
    __shared__ int64_t sh[LIST_THREADS / 64];
    const int t = threadIdx.x;
    int nn[2];
    int64_t sA = 0, sL = 0, sc[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = 2 * t + q;
        nn[q] = (i < a.count) ? (int)a.n[i] : 0;
        sA += (int64_t)nn[q] * nn[q];
        sL += nn[q];
        if (nn[q] > 0) sc[class_of(nn[q])] += 1;
    }
    int64_t tot;
    int64_t eA = block_scan_excl(sA, sh, tot);
    int64_t eL = block_scan_excl(sL, sh, tot);
    int64_t ec[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) ec[c] = block_scan_excl(sc[c], sh, tot);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = 2 * t + q;
        if (i >= a.count) continue;
        const int n = nn[q], c = class_of(n);
        WorkItem w;
        w.offA = a.offA0 + eA;
        w.offL = a.offL0 + eL;
        w.n = n;
        w.idx = a.b0 + i;
        items[a.cls_base[c] + ec[c]] = w;
        eA += (int64_t)n * n;
        eL += n;
        ec[c] += 1;
    }
}

// Device address of `scratch` on each device, formed once per device (host
// code must not use the array's name as an address).
static std::mutex g_mu;
static void *g_ptr[64];

static bed_status scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(BED_ERR_UNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BED_OK;
}

}  // namespace bed

using namespace bed;

extern "C" bed_status bed_syevd_noalloc(bed_dtype dt, int64_t batch, const int32_t *n,
                                        const void *A, void *lambda, void *Q, int32_t *info,
                                        void *stream)
{
    bed_status st = check_sizes(dt, batch, n);
    if (st != BED_OK) return st;
    if (batch == 0) return BED_OK;
    if (batch > NOALLOC_MAX)
        return fail(BED_ERR_INVALID_ARG, "batch %lld exceeds the allocation-free maximum %d",
                    (long long)batch, NOALLOC_MAX);
    if ((st = check_ptr(A, dt, "A", false)) != BED_OK) return st;
    if ((st = check_ptr(lambda, dt, "lambda", false)) != BED_OK) return st;
    if ((st = check_ptr(Q, dt, "Q", false)) != BED_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bed_tune dflt = default_tune();
    bool uniform = true;
    int cnt[3] = {0, 0, 0};
    for (int64_t b = 0; b < batch; ++b) {
        uniform = uniform && n[b] == n[0];
        cnt[size_class(n[b])] += 1;
    }
    if (uniform) {  // one workgroup per matrix, offsets formed in the kernel
        hipError_t e = launch_uniform(dt, class_shape(size_class(n[0]), dflt), A, n[0], batch,
                                      lambda, Q, info, s);
        return e == hipSuccess ? BED_OK : hip_fail(e, "kernel launch");
    }
    void *base = nullptr;
    if ((st = scratch_ptr(&base)) != BED_OK) return st;
    WorkItem *items = (WorkItem *)base;
    // class segments: [0, cnt0), [cnt0, cnt0 + cnt1), [cnt0 + cnt1, batch)
    const int seg[3] = {0, cnt[0], cnt[0] + cnt[1]};
    ChunkArgs a;
    int64_t offA = 0, offL = 0;
    int done[3] = {0, 0, 0};
    for (int64_t b0 = 0; b0 < batch; b0 += CHUNK) {
        const int m = (int)std::min<int64_t>(CHUNK, batch - b0);
        a.offA0 = offA;
        a.offL0 = offL;
        a.b0 = (int32_t)b0;
        a.count = m;
        for (int c = 0; c < 3; ++c) a.cls_base[c] = seg[c] + done[c];
        for (int i = 0; i < m; ++i) {
            const int v = n[b0 + i];
            a.n[i] = (uint8_t)v;
            offA += (int64_t)v * v;
            offL += v;
            done[size_class(v)] += 1;
        }
        hipLaunchKernelGGL(k_noalloc_list, dim3(1), dim3(LIST_THREADS), 0, s, a, items);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "work-list launch");
    }
    for (int c = 2; c >= 0; --c) {  // largest class first
        if (cnt[c] == 0) continue;
        hipError_t e = launch_list(dt, class_shape(c, dflt), A, lambda, Q, info, items + seg[c],
                                   cnt[c], nullptr, cnt[c], s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return BED_OK;
}
