// bed_api.cpp -- C ABI: validation, plans (size classes, work lists, launch
// schedule), the convenience plan cache and status strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bed.h"
#include "bed_internal.hpp"
#include "bed_host.hpp"
#include "bed_lru.hpp"

using namespace bed;

namespace bed {

static thread_local std::string g_last_error;

bed_status fail(bed_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

bed_status hip_fail(hipError_t e, const char *what)
{
    return fail(BED_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t dtype_size(bed_dtype dt) { return dt == BED_F64 ? 8 : 4; }

bed_status check_sizes(bed_dtype dt, int64_t batch, const int32_t *n, int nmax)
{
    if (dt != BED_F32 && dt != BED_F64) return fail(BED_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
    if (batch < 0) return fail(BED_ERR_INVALID_ARG, "batch < 0");
    if (batch > 0 && n == nullptr) return fail(BED_ERR_INVALID_ARG, "n is NULL");
    if (batch > (int64_t)INT32_MAX) return fail(BED_ERR_INVALID_ARG, "batch too large");
    for (int64_t b = 0; b < batch; ++b) {
        if (n[b] < 1) return fail(BED_ERR_INVALID_ARG, "n[%lld] = %d < 1", (long long)b, n[b]);
        if (n[b] > nmax)
            return fail(BED_ERR_UNSUPPORTED, "n[%lld] = %d > %d is not supported here",
                        (long long)b, n[b], nmax);
    }
    return BED_OK;
}

bed_status check_ptr(const void *p, bed_dtype dt, const char *name, bool nullable)
{
    if (p == nullptr) {
        if (nullable) return BED_OK;
        return fail(BED_ERR_INVALID_ARG, "%s is NULL", name);
    }
    if (((uintptr_t)p) % dtype_size(dt) != 0)
        return fail(BED_ERR_INVALID_ARG, "%s is not %zu-byte aligned", name, dtype_size(dt));
    return BED_OK;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

int device_cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}

int size_class(int n) { return n <= 16 ? 0 : (n <= 32 ? 1 : 2); }

TeamShape class_shape(int cls, const bed_tune &t)
{
    switch (cls) {
    case 0: return TeamShape{16, 64, t.leaf > 0 ? t.leaf : leaf_default(16)};
    case 1: return TeamShape{32, t.threads_mid > 0 ? t.threads_mid : 128,
                             t.leaf > 0 ? t.leaf : leaf_default(32)};
    default: return TeamShape{64, t.threads_big > 0 ? t.threads_big : 512,
                              t.leaf > 0 ? t.leaf : leaf_default(64)};
    }
}

bed_tune default_tune()
{
    bed_tune t;
    t.threads_big = 512;
    t.threads_mid = 256;
    t.waves_per_cu = 0;
    t.order = 0;
    t.persistent = 0;
    t.leaf = 0;  // per size class
    return t;
}

}  // namespace bed

// ------------------------------------------------------------------ plans
struct bed_plan {
    bed_dtype dt;
    int64_t batch;
    bed_tune tune;
    bool uniform;  // all n equal: one launch, offsets computed in-kernel
    int n0;
    // per size class: device work list and persistent counters
    struct Cls {
        TeamShape ts;
        int count = 0;
        int grid = 0;
        WorkItem *d_items = nullptr;
        int *d_counter = nullptr;
    } cls[3];
    std::vector<int32_t> n;
};

static void plan_free_device(bed_plan *p)
{
    for (auto &c : p->cls) {
        if (c.d_items) (void)hipFree(c.d_items);
        if (c.d_counter) (void)hipFree(c.d_counter);
        c.d_items = nullptr;
        c.d_counter = nullptr;
    }
}

static bed_status plan_build(bed_plan *p, bed_dtype dt, int64_t batch, const int32_t *n,
                             const bed_tune &tune)
{
    p->dt = dt;
    p->batch = batch;
    p->tune = tune;
    p->n.assign(n, n + batch);
    p->uniform = batch > 0 && std::all_of(n, n + batch, [&](int32_t v) { return v == n[0]; });
    p->n0 = batch > 0 ? n[0] : 0;
    for (int c = 0; c < 3; ++c) p->cls[c].ts = class_shape(c, tune);
    if (p->uniform && !tune.persistent) {
        const int c = size_class(p->n0);
        p->cls[c].count = (int)batch;
        return BED_OK;
    }
    std::vector<WorkItem> items[3];
    int64_t offA = 0, offL = 0;
    for (int64_t b = 0; b < batch; ++b) {
        WorkItem w{offA, offL, n[b], (int32_t)b};
        items[size_class(n[b])].push_back(w);
        offA += (int64_t)n[b] * n[b];
        offL += n[b];
    }
    const int cus = device_cu_count();
    for (int c = 0; c < 3; ++c) {
        auto &v = items[c];
        if (v.empty()) continue;
        if (tune.order == 0)  // LPT: largest matrices first
            std::stable_sort(v.begin(), v.end(),
                             [](const WorkItem &x, const WorkItem &y) { return x.n > y.n; });
        auto &C = p->cls[c];
        C.count = (int)v.size();
        hipError_t e = hipMalloc(&C.d_items, sizeof(WorkItem) * v.size());
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(work list)");
        e = hipMemcpy(C.d_items, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(work list)");
        if (tune.persistent) {
            e = hipMalloc(&C.d_counter, 2 * sizeof(int));
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(counter)");
            e = hipMemset(C.d_counter, 0, 2 * sizeof(int));
            if (e != hipSuccess) return hip_fail(e, "hipMemset(counter)");
            int per_cu = tune.waves_per_cu > 0
                             ? std::max(1, tune.waves_per_cu / (C.ts.nt / 64))
                             : blocks_per_cu(dt, C.ts);
            C.grid = std::min(C.count, std::max(1, per_cu * cus));
        } else {
            C.grid = C.count;
        }
    }
    return BED_OK;
}

extern "C" bed_status bed_plan_create(bed_plan **plan, bed_dtype dt, int64_t batch,
                                      const int32_t *n, const bed_tune *tune, void *stream)
{
    if (!plan) return fail(BED_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    bed_status st = check_sizes(dt, batch, n);
    if (st != BED_OK) return st;
    if (stream_capturing((hipStream_t)stream))
        return fail(BED_ERR_CAPTURE, "bed_plan_create while its stream is being captured");
    bed_tune t = tune ? *tune : tuned_or_default(dt, batch, n);
    const bed_tune dflt = default_tune();
    if (t.threads_big == 0) t.threads_big = dflt.threads_big;
    if (t.threads_mid == 0) t.threads_mid = dflt.threads_mid;
    if (t.leaf != 0 && !leaf_supported(t.leaf))
        return fail(BED_ERR_INVALID_ARG, "unsupported leaf size %d (2, 4 or 8)", t.leaf);
    if (!team_supported(dt, TeamShape{64, t.threads_big}) ||
        !team_supported(dt, TeamShape{32, t.threads_mid}))
        return fail(BED_ERR_INVALID_ARG, "unsupported thread counts (%d, %d)", t.threads_big,
                    t.threads_mid);
    auto *p = new (std::nothrow) bed_plan();
    if (!p) return fail(BED_ERR_NOMEM, "host allocation failed");
    st = plan_build(p, dt, batch, n, t);
    if (st != BED_OK) {
        plan_free_device(p);
        delete p;
        return st;
    }
    *plan = p;
    return BED_OK;
}

namespace bed {
bed_status plan_run_impl(const bed_plan *p, const void *A, void *lam, void *Q, int32_t *info,
                         hipStream_t s)
{
    if (p->uniform && !p->tune.persistent) {
        const int c = size_class(p->n0);
        hipError_t e = launch_uniform(p->dt, p->cls[c].ts, A, p->n0, p->batch, lam, Q, info, s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return BED_OK;
    }
    // largest class first so its long-running teams start early
    for (int c = 2; c >= 0; --c) {
        const auto &C = p->cls[c];
        if (C.count == 0) continue;
        hipError_t e = launch_list(p->dt, C.ts, A, lam, Q, info, C.d_items, C.count, C.d_counter,
                                   C.grid, s);
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return BED_OK;
}
}  // namespace bed

extern "C" bed_status bed_plan_run(const bed_plan *plan, const void *A, void *lambda, void *Q,
                                   int32_t *info, void *stream)
{
    if (!plan) return fail(BED_ERR_INVALID_ARG, "plan is NULL");
    if (plan->batch == 0) return BED_OK;
    bed_status st;
    if ((st = check_ptr(A, plan->dt, "A", false)) != BED_OK) return st;
    if ((st = check_ptr(lambda, plan->dt, "lambda", false)) != BED_OK) return st;
    if ((st = check_ptr(Q, plan->dt, "Q", true)) != BED_OK) return st;
    return plan_run_impl(plan, A, lambda, Q, info, (hipStream_t)stream);
}

extern "C" bed_status bed_plan_get_tune(const bed_plan *plan, bed_tune *out)
{
    if (!plan || !out) return fail(BED_ERR_INVALID_ARG, "NULL argument");
    *out = plan->tune;
    return BED_OK;
}

extern "C" void bed_plan_destroy(bed_plan *plan)
{
    if (!plan) return;
    plan_free_device(plan);
    delete plan;
}

// ------------------------------------------------------------------ plan cache
// bed_syevd / bed_syevals keep one plan per (dtype, n[], stream): a persistent
// plan's work counter is then never shared by launches on two streams.  The
// cache holds at most PLAN_CACHE_MAX plans; an evicted plan is freed after the
// event recorded behind its last launch has completed.  A plan used while its
// stream is being captured is pinned: the graph holds its device pointers.
namespace {
struct CacheKey {
    bed_dtype dt;
    void *stream;
    std::vector<int32_t> n;
    bool operator<(const CacheKey &o) const
    {
        if (dt != o.dt) return dt < o.dt;
        if (stream != o.stream) return stream < o.stream;
        return n < o.n;
    }
};
struct CachedPlan {
    bed_plan *plan = nullptr;
    hipEvent_t last = nullptr;  // recorded after the latest (uncaptured) launch
};
constexpr size_t PLAN_CACHE_MAX = 32;
std::mutex g_cache_mu;
Lru<CacheKey, CachedPlan> g_cache(PLAN_CACHE_MAX);

void release_cached(CachedPlan &c)
{
    if (c.last) {
        (void)hipEventSynchronize(c.last);
        (void)hipEventDestroy(c.last);
    }
    bed_plan_destroy(c.plan);
}
}  // namespace

static bed_status solve(bed_dtype dt, int64_t batch, const int32_t *n, const void *A, void *lambda,
                        void *Q, int32_t *info, void *stream, bool want_q)
{
    bed_status st = check_sizes(dt, batch, n, NMAX_BIG);
    if (st != BED_OK) return st;
    if (batch == 0) return BED_OK;
    const bool uniform = std::all_of(n, n + batch, [&](int32_t v) { return v == n[0]; });
    const bool big = std::any_of(n, n + batch, [](int32_t v) { return v > 64; });
    if (big && !uniform)
        return fail(BED_ERR_UNSUPPORTED, "n > 64 is supported in uniform batches only");
    if (big && dt != BED_F32)
        return fail(BED_ERR_UNSUPPORTED, "n = %d > 64 is supported in binary32 only", n[0]);
    if ((st = check_ptr(A, dt, "A", false)) != BED_OK) return st;
    if ((st = check_ptr(lambda, dt, "lambda", false)) != BED_OK) return st;
    if (want_q && (st = check_ptr(Q, dt, "Q", false)) != BED_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (big) return big_solve(dt, batch, n[0], A, lambda, want_q ? Q : nullptr, info, s);
    if (uniform) {
        // no descriptor needed: one workgroup per matrix, offsets in-kernel
        bed_tune t = tuned_or_default(dt, batch, n);
        TeamShape ts = class_shape(size_class(n[0]), t);
        if (!t.persistent) {
            hipError_t e = launch_uniform(dt, ts, A, n[0], batch, lambda, want_q ? Q : nullptr,
                                          info, s);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
            return BED_OK;
        }
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    const bool capturing = stream_capturing(s);
    CacheKey key{dt, stream, std::vector<int32_t>(n, n + batch)};
    CachedPlan *c = g_cache.find(key);
    if (!c) {
        if (capturing)
            return fail(BED_ERR_CAPTURE, "first bed_syevd for a new size mix during capture");
        CachedPlan fresh;
        st = bed_plan_create(&fresh.plan, dt, batch, n, nullptr, stream);
        if (st != BED_OK) return st;
        hipError_t e = hipEventCreateWithFlags(&fresh.last, hipEventDisableTiming);
        if (e != hipSuccess) {
            bed_plan_destroy(fresh.plan);
            return hip_fail(e, "hipEventCreate");
        }
        for (CachedPlan &old : g_cache.insert(key, fresh)) release_cached(old);
        c = g_cache.find(key);
    }
    st = plan_run_impl(c->plan, A, lambda, want_q ? Q : nullptr, info, s);
    if (st != BED_OK) return st;
    if (capturing) {
        g_cache.pin(key);
    } else {
        hipError_t e = hipEventRecord(c->last, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    return BED_OK;
}

extern "C" int32_t bed_cache_entries(void)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return (int32_t)g_cache.size();
}

extern "C" bed_status bed_syevd(bed_dtype dt, int64_t batch, const int32_t *n, const void *A,
                                void *lambda, void *Q, int32_t *info, void *stream)
{
    return solve(dt, batch, n, A, lambda, Q, info, stream, true);
}

extern "C" bed_status bed_syevals(bed_dtype dt, int64_t batch, const int32_t *n, const void *A,
                                  void *lambda, int32_t *info, void *stream)
{
    return solve(dt, batch, n, A, lambda, nullptr, info, stream, false);
}

extern "C" const char *bed_status_string(bed_status st)
{
    switch (st) {
    case BED_OK: return "BED_OK";
    case BED_ERR_INVALID_ARG: return "BED_ERR_INVALID_ARG";
    case BED_ERR_UNSUPPORTED: return "BED_ERR_UNSUPPORTED";
    case BED_ERR_HIP: return "BED_ERR_HIP";
    case BED_ERR_NOMEM: return "BED_ERR_NOMEM";
    case BED_ERR_CAPTURE: return "BED_ERR_CAPTURE";
    case BED_ERR_BUSY: return "BED_ERR_BUSY";
    }
    return "BED_ERR_UNKNOWN";
}

extern "C" const char *bed_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t bed_version(void) { return 100; }
