// bed_tune.cpp -- autotuner for plan schedules.
//
// A schedule (bed_tune) picks, per size mix: the team size of the n > 32 and
// 16 < n <= 32 classes, persistent vs. one-workgroup-per-matrix launches, the
// list order and the leaf cutoff of the divide step (Sec. 2.2: leaves of at
// most 2, 4 or 8 elements, solved by Jacobi).  Candidates are timed with HIP events on the caller's
// stream; the winner is cached per (device arch, dtype, histogram of n) in
// the process and, when BED_TUNE_CACHE names a file, in that JSON file.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bed_host.hpp"

using namespace bed;

namespace {

std::mutex g_mu;
std::map<std::string, bed_tune> g_tuned;
bool g_file_loaded = false;

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string tune_key(bed_dtype dt, int64_t batch, const int32_t *n)
{
    int64_t hist[65] = {0};
    for (int64_t b = 0; b < batch; ++b) hist[n[b]]++;
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the histogram
    for (int i = 1; i <= 64; ++i) {
        uint64_t v = (uint64_t)hist[i];
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    }
    char buf[128];
    snprintf(buf, sizeof buf, "%s|%s|%lld|%016llx", arch_name().c_str(),
             dt == BED_F64 ? "f64" : "f32", (long long)batch, (unsigned long long)h);
    return buf;
}

void load_file_locked()
{
    if (g_file_loaded) return;
    g_file_loaded = true;
    const char *path = getenv("BED_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char key[256];
        bed_tune t = default_tune();
        const int got = sscanf(line, " \"%255[^\"]\" : [ %d , %d , %d , %d , %d , %d ]", key,
                               &t.threads_big, &t.threads_mid, &t.waves_per_cu, &t.order,
                               &t.persistent, &t.leaf);
        if (got >= 6 && (t.leaf == 0 || leaf_supported(t.leaf))) g_tuned[key] = t;
    }
    fclose(f);
}

void save_file_locked()
{
    const char *path = getenv("BED_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : g_tuned) {
        const bed_tune &t = kv.second;
        fprintf(f, "  \"%s\" : [ %d , %d , %d , %d , %d , %d ]%s\n", kv.first.c_str(),
                t.threads_big, t.threads_mid, t.waves_per_cu, t.order, t.persistent, t.leaf,
                ++i < g_tuned.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
}

}  // namespace

namespace bed {
bed_tune tuned_or_default(bed_dtype dt, int64_t batch, const int32_t *n)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    if (!g_tuned.empty()) {
        auto it = g_tuned.find(tune_key(dt, batch, n));
        if (it != g_tuned.end()) return it->second;
    }
    return default_tune();
}
}  // namespace bed

extern "C" bed_status bed_autotune(bed_dtype dt, int64_t batch, const int32_t *n, const void *A,
                                   void *lambda, void *Q, void *stream, bed_tune *out)
{
    bed_status st = check_sizes(dt, batch, n);
    if (st != BED_OK) return st;
    if (batch == 0) return fail(BED_ERR_INVALID_ARG, "autotune of an empty batch");
    hipStream_t s = (hipStream_t)stream;
    if (stream_capturing(s)) return fail(BED_ERR_CAPTURE, "autotune during stream capture");
    std::vector<bed_tune> cands;
    for (int tb : {128, 256, 512})
        for (int tm : {64, 128, 256})
            for (int pers : {0, 1}) {
                bed_tune t;
                t.threads_big = tb;
                t.threads_mid = tm;
                t.waves_per_cu = 0;
                t.order = 0;
                t.persistent = pers;
                t.leaf = 0;
                cands.push_back(t);
            }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(BED_ERR_HIP, "hipEventCreate failed");
    float best_ms = 1e30f;
    bed_tune best = default_tune();
    auto trial = [&](const bed_tune &t) {
        bed_plan *p = nullptr;
        if (bed_plan_create(&p, dt, batch, n, &t, stream) != BED_OK) return;
        bool ok = true;
        for (int w = 0; w < 2 && ok; ++w) ok = plan_run_impl(p, A, lambda, Q, nullptr, s) == BED_OK;
        const int reps = 5;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && ok; ++r) ok = plan_run_impl(p, A, lambda, Q, nullptr, s) == BED_OK;
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (ok && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
            ms /= reps;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        (void)hipStreamSynchronize(s);
        bed_plan_destroy(p);
    };
    for (const bed_tune &t : cands) trial(t);
    // then the leaf cutoff, with the best team shapes and launch form
    const bed_tune shape = best;
    for (int leaf : {2, 4, 8}) {
        bed_tune t = shape;
        t.leaf = leaf;
        trial(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_file_locked();
        g_tuned[tune_key(dt, batch, n)] = best;
        save_file_locked();
    }
    if (out) *out = best;
    return BED_OK;
}

extern "C" bed_status bed_tune_set(bed_dtype dt, int64_t batch, const int32_t *n,
                                   const bed_tune *tune)
{
    bed_status st = check_sizes(dt, batch, n);
    if (st != BED_OK) return st;
    if (!tune) return fail(BED_ERR_INVALID_ARG, "tune is NULL");
    bed_tune t = *tune;
    const bed_tune dflt = default_tune();
    if (t.threads_big == 0) t.threads_big = dflt.threads_big;
    if (t.threads_mid == 0) t.threads_mid = dflt.threads_mid;
    if (t.leaf != 0 && !leaf_supported(t.leaf))
        return fail(BED_ERR_INVALID_ARG, "unsupported leaf size %d (2, 4 or 8)", t.leaf);
    if (!team_supported(dt, TeamShape{64, t.threads_big}) ||
        !team_supported(dt, TeamShape{32, t.threads_mid}))
        return fail(BED_ERR_INVALID_ARG, "unsupported thread counts (%d, %d)", t.threads_big,
                    t.threads_mid);
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    g_tuned[tune_key(dt, batch, n)] = t;
    return BED_OK;
}
