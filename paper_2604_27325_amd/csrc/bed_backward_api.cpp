// bed_backward_api.cpp -- C ABI of the backward kernel, and the cached work
// lists of mixed-size batches that it shares with the spectral functions.
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "bed_host.hpp"
#include "bed_lru.hpp"

using namespace bed;

namespace {
// Work lists of mixed-size batches, one per (dtype, n[], stream), at most
// BWD_CACHE_MAX of them (least recently used evicted after the event behind
// its last launch has completed; pinned once used under graph capture).
struct BwdKey {
    int dt;
    void *stream;
    std::vector<int32_t> n;
    bool operator<(const BwdKey &o) const
    {
        if (dt != o.dt) return dt < o.dt;
        if (stream != o.stream) return stream < o.stream;
        return n < o.n;
    }
};
struct BwdPlan {
    WorkItem *d_items = nullptr;
    int count = 0;
    int nmax = 64;
    hipEvent_t last = nullptr;
};
constexpr size_t BWD_CACHE_MAX = 32;
std::mutex g_bwd_mu;
Lru<BwdKey, BwdPlan> g_bwd_cache(BWD_CACHE_MAX);

void release_bwd(BwdPlan &p)
{
    if (p.last) {
        (void)hipEventSynchronize(p.last);
        (void)hipEventDestroy(p.last);
    }
    if (p.d_items) (void)hipFree(p.d_items);
}
}  // namespace

namespace bed {
// Runs `launch` with the device work list (packed offsets in input order) of
// a mixed-size batch, taken from the bounded per-stream cache (created on
// first use, refused under capture), and records the cache entry's event
// behind the launch (or pins the entry when the stream is being captured).
bed_status with_worklist(bed_dtype dt, int64_t batch, const int32_t *n, hipStream_t s,
                         const std::function<hipError_t(const WorkItem *, int, int)> &launch)
{
    std::lock_guard<std::mutex> lk(g_bwd_mu);
    const bool capturing = stream_capturing(s);
    BwdKey key{(int)dt, (void *)s, std::vector<int32_t>(n, n + batch)};
    BwdPlan *p = g_bwd_cache.find(key);
    if (!p) {
        if (capturing)
            return fail(BED_ERR_CAPTURE, "first call for a new size mix during capture");
        std::vector<WorkItem> items;
        int64_t offA = 0, offL = 0;
        for (int64_t b = 0; b < batch; ++b) {
            items.push_back(WorkItem{offA, offL, n[b], (int32_t)b});
            offA += (int64_t)n[b] * n[b];
            offL += n[b];
        }
        BwdPlan fresh;
        fresh.nmax = *std::max_element(n, n + batch);
        fresh.count = (int)batch;
        hipError_t e = hipMalloc(&fresh.d_items, sizeof(WorkItem) * items.size());
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(work list)");
        e = hipMemcpy(fresh.d_items, items.data(), sizeof(WorkItem) * items.size(),
                      hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fresh.last, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipFree(fresh.d_items);
            return hip_fail(e, "work list");
        }
        for (BwdPlan &old : g_bwd_cache.insert(key, fresh)) release_bwd(old);
        p = g_bwd_cache.find(key);
    }
    hipError_t e = launch(p->d_items, p->count, p->nmax);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (capturing) {
        g_bwd_cache.pin(key);
    } else {
        e = hipEventRecord(p->last, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    return BED_OK;
}
}  // namespace bed

extern "C" bed_status bed_syevd_backward(bed_dtype dt, int64_t batch, const int32_t *n,
                                         const void *lambda, const void *Q, const void *dlambda,
                                         const void *dQ, void *dA, double degeneracy_eps,
                                         void *stream)
{
    bed_status st = check_sizes(dt, batch, n);
    if (st != BED_OK) return st;
    if (batch == 0) return BED_OK;
    if ((st = check_ptr(lambda, dt, "lambda", false)) != BED_OK) return st;
    if ((st = check_ptr(Q, dt, "Q", false)) != BED_OK) return st;
    if ((st = check_ptr(dlambda, dt, "dlambda", true)) != BED_OK) return st;
    if ((st = check_ptr(dQ, dt, "dQ", true)) != BED_OK) return st;
    if ((st = check_ptr(dA, dt, "dA", false)) != BED_OK) return st;
    const double eps = degeneracy_eps > 0 ? degeneracy_eps
                                          : 1e3 * (dt == BED_F32 ? 0x1p-24 : 0x1p-53);
    hipStream_t s = (hipStream_t)stream;
    const bool uniform = std::all_of(n, n + batch, [&](int32_t v) { return v == n[0]; });
    if (uniform) {
        hipError_t e = launch_backward_uniform(dt, n[0], lambda, Q, dlambda, dQ, dA, n[0], batch,
                                               eps, s);
        return e == hipSuccess ? BED_OK : hip_fail(e, "backward launch");
    }
    return with_worklist(dt, batch, n, s, [&](const WorkItem *items, int count, int nmax) {
        return launch_backward(dt, nmax, lambda, Q, dlambda, dQ, dA, items, count, eps, s);
    });
}
