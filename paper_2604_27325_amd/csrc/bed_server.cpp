// bed_server.cpp -- continuous-batching request server.
//
// Requests (count matrices of one size n, caller-owned device buffers) are
// admitted while the in-flight matrix count and the admitted bytes stay under
// the configured limits (bed_admit.hpp).  At admission an event is recorded on
// the caller's stream, so the step that reads a request's A first waits for
// the work the caller enqueued before submitting (the kernel or copy that
// produced A).  A scheduler thread packs every admitted, not-yet-launched
// request into one step on a free stream (up to max_step matrices), uploads
// the step's pointer work list from pinned host memory into a device buffer
// owned by that stream slot, launches one kernel per size class and records
// an event.  Steps on different streams overlap on the
// device; completion is observed by polling the events.  The per-matrix
// kernel configuration depends only on (n, dtype), so each request's result is
// bitwise the same alone or in any mix.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <algorithm>
#include <thread>
#include <vector>

#include "bed_admit.hpp"
#include "bed_host.hpp"

using namespace bed;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket;
    bed_dtype dt;
    int32_t count, n;
    const void *A;
    void *lam, *Q;
    int32_t *info;
    int64_t bytes;
    hipEvent_t ready;  // recorded on the caller's stream at submission
    hipStream_t producer;
    Clock::time_point t_submit;
    bool launched = false, done = false;
    double latency_us = 0.0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    PtrItem *h_items = nullptr;  // pinned staging
    PtrItem *d_items = nullptr;  // device work list
    bool busy = false;
    std::vector<uint64_t> tickets;
};

}  // namespace

struct bed_server {
    bed_server_opts opts;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<uint64_t> pending;
    std::map<uint64_t, Request> reqs;
    std::vector<hipEvent_t> free_events;  // recycled readiness events
    uint64_t next_ticket = 1;
    Admission adm;
    bool stop = false;
    std::thread worker;
    int device = 0;
    std::string error;
};

static void server_loop(bed_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        // completions
        bool progressed = false;
        for (auto &sl : s->slots) {
            if (!sl.busy) continue;
            if (hipEventQuery(sl.done_ev) == hipSuccess) {
                const auto now = Clock::now();
                for (uint64_t tk : sl.tickets) {
                    auto it = s->reqs.find(tk);
                    if (it == s->reqs.end()) continue;
                    Request &r = it->second;
                    r.done = true;
                    r.latency_us =
                        std::chrono::duration<double, std::micro>(now - r.t_submit).count();
                    s->adm.release(r.count, r.bytes);
                    s->free_events.push_back(r.ready);
                    r.ready = nullptr;
                }
                sl.tickets.clear();
                sl.busy = false;
                progressed = true;
            }
        }
        if (progressed) s->cv_done.notify_all();
        // launches: every pending request goes into the next step on a free slot
        Slot *free_slot = nullptr;
        for (auto &sl : s->slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        if (free_slot && !s->pending.empty()) {
            Slot &sl = *free_slot;
            int nitems = 0;
            std::vector<PtrItem> cls_items[2][3];  // [dtype][size class]
            while (!s->pending.empty()) {
                const uint64_t tk = s->pending.front();
                Request &r = s->reqs[tk];
                if (nitems > 0 && nitems + r.count > s->opts.max_step) break;
                s->pending.pop_front();
                const size_t es = dtype_size(r.dt);
                for (int32_t i = 0; i < r.count; ++i) {
                    PtrItem it;
                    it.A = (const char *)r.A + (size_t)i * r.n * r.n * es;
                    it.lam = (char *)r.lam + (size_t)i * r.n * es;
                    it.Q = (char *)r.Q + (size_t)i * r.n * r.n * es;
                    it.info = r.info ? r.info + i : nullptr;
                    it.n = r.n;
                    cls_items[r.dt == BED_F64][size_class(r.n)].push_back(it);
                }
                nitems += r.count;
                r.launched = true;
                sl.tickets.push_back(tk);
            }
            // every request's input is complete on its producer stream first:
            // per producer stream, the event of its latest request covers the
            // earlier ones (work on one stream completes in order)
            hipError_t e = hipSuccess;
            std::map<hipStream_t, uint64_t> latest;
            for (uint64_t tk : sl.tickets) {
                auto &v = latest[s->reqs[tk].producer];
                v = std::max(v, tk);
            }
            for (const auto &kv : latest)
                if (e == hipSuccess) e = hipStreamWaitEvent(sl.stream, s->reqs[kv.second].ready, 0);
            // stage the list in pinned memory grouped by (dtype, class)
            int off = 0;
            struct Launch {
                bed_dtype dt;
                int cls, off, count;
            };
            std::vector<Launch> launches;
            for (int d = 0; d < 2; ++d)
                for (int c = 2; c >= 0; --c) {
                    auto &v = cls_items[d][c];
                    if (v.empty()) continue;
                    std::copy(v.begin(), v.end(), sl.h_items + off);
                    launches.push_back(Launch{d ? BED_F64 : BED_F32, c, off, (int)v.size()});
                    off += (int)v.size();
                }
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.d_items, sl.h_items, sizeof(PtrItem) * off,
                                   hipMemcpyHostToDevice, sl.stream);
            const bed_tune dflt = default_tune();
            for (const Launch &L : launches)
                if (e == hipSuccess)
                    e = launch_ptrlist(L.dt, class_shape(L.cls, dflt), sl.d_items + L.off, L.count,
                                       sl.stream);
            if (e == hipSuccess) e = hipEventRecord(sl.done_ev, sl.stream);
            if (e != hipSuccess) s->error = hipGetErrorString(e);
            sl.busy = true;
            continue;
        }
        if (s->stop && s->pending.empty()) {
            bool any = false;
            for (auto &sl : s->slots) any |= sl.busy;
            if (!any) break;
        }
        // idle: wait for a submission, or poll in-flight events shortly
        bool any_busy = false;
        for (auto &sl : s->slots) any_busy |= sl.busy;
        if (any_busy)
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        else
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
    }
}

extern "C" bed_status bed_server_create(bed_server **out, const bed_server_opts *o)
{
    if (!out) return fail(BED_ERR_INVALID_ARG, "server is NULL");
    *out = nullptr;
    bed_server_opts opts{};
    if (o) opts = *o;
    if (opts.streams <= 0) opts.streams = 4;
    if (opts.streams > 16) return fail(BED_ERR_INVALID_ARG, "streams must be 1..16");
    if (opts.max_step <= 0) opts.max_step = 4096;
    auto *s = new (std::nothrow) bed_server();
    if (!s) return fail(BED_ERR_NOMEM, "host allocation failed");
    s->opts = opts;
    s->adm.max_mats = opts.max_inflight;
    s->adm.max_bytes = opts.mem_budget;
    s->device = opts.device;
    if (hipSetDevice(s->device) != hipSuccess) {
        delete s;
        return fail(BED_ERR_HIP, "hipSetDevice(%d) failed", opts.device);
    }
    s->slots.resize(opts.streams);
    for (auto &sl : s->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&sl.h_items, sizeof(PtrItem) * opts.max_step * 2, 0);
        if (e == hipSuccess) e = hipMalloc(&sl.d_items, sizeof(PtrItem) * opts.max_step * 2);
        if (e != hipSuccess) {
            bed_server_destroy(s);
            return hip_fail(e, "server resources");
        }
    }
    s->worker = std::thread(server_loop, s);
    *out = s;
    return BED_OK;
}

extern "C" bed_status bed_server_submit(bed_server *s, bed_dtype dt, int32_t count, int32_t n,
                                        const void *A, void *lambda, void *Q, int32_t *info,
                                        void *stream, uint64_t *ticket)
{
    if (!s || !ticket) return fail(BED_ERR_INVALID_ARG, "NULL argument");
    if (count < 1) return fail(BED_ERR_INVALID_ARG, "count < 1");
    if (count > s->opts.max_step) return fail(BED_ERR_INVALID_ARG, "count > max_step");
    int32_t nn = n;
    bed_status st = check_sizes(dt, 1, &nn);
    if (st != BED_OK) return st;
    if ((st = check_ptr(A, dt, "A", false)) != BED_OK) return st;
    if ((st = check_ptr(lambda, dt, "lambda", false)) != BED_OK) return st;
    if ((st = check_ptr(Q, dt, "Q", false)) != BED_OK) return st;
    const int64_t bytes = request_bytes(count, n, dtype_size(dt));
    std::lock_guard<std::mutex> lk(s->mu);
    hipEvent_t ev = nullptr;
    if (!s->free_events.empty()) {
        ev = s->free_events.back();
        s->free_events.pop_back();
    } else {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    switch (s->adm.admit(count, bytes)) {
    case ADMIT_OK: break;
    case ADMIT_INFLIGHT:
        s->free_events.push_back(ev);
        return fail(BED_ERR_BUSY, "in-flight matrix limit reached");
    case ADMIT_MEMORY:
        s->free_events.push_back(ev);
        return fail(BED_ERR_BUSY, "memory budget reached");
    }
    hipError_t e = hipEventRecord(ev, (hipStream_t)stream);
    if (e != hipSuccess) {
        s->adm.release(count, bytes);
        s->free_events.push_back(ev);
        return hip_fail(e, "hipEventRecord on the submitting stream");
    }
    Request r;
    r.ticket = s->next_ticket++;
    r.dt = dt;
    r.count = count;
    r.n = n;
    r.A = A;
    r.lam = lambda;
    r.Q = Q;
    r.info = info;
    r.bytes = bytes;
    r.ready = ev;
    r.producer = (hipStream_t)stream;
    r.t_submit = Clock::now();
    s->reqs.emplace(r.ticket, r);
    s->pending.push_back(r.ticket);
    *ticket = r.ticket;
    s->cv.notify_all();
    return BED_OK;
}

extern "C" bed_status bed_server_poll(bed_server *s, uint64_t ticket, int32_t *done,
                                      double *latency_us)
{
    if (!s || !done) return fail(BED_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->error.empty()) return fail(BED_ERR_HIP, "server: %s", s->error.c_str());
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(BED_ERR_INVALID_ARG, "unknown ticket %llu",
                                         (unsigned long long)ticket);
    *done = it->second.done ? 1 : 0;
    if (latency_us) *latency_us = it->second.latency_us;
    if (it->second.done) s->reqs.erase(it);
    return BED_OK;
}

extern "C" bed_status bed_server_drain(bed_server *s)
{
    if (!s) return fail(BED_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->adm.idle() || !s->error.empty(); });
    if (!s->error.empty()) return fail(BED_ERR_HIP, "server: %s", s->error.c_str());
    return BED_OK;
}

extern "C" void bed_server_destroy(bed_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
        if (sl.h_items) (void)hipHostFree(sl.h_items);
        if (sl.d_items) (void)hipFree(sl.d_items);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
}
