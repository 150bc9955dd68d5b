// Continuous-batching request loop on one GPU.
//
// Requests (float32 host series of power-of-two lengths) are copied into
// pinned host staging on fdas_submit and queued.  One scheduler thread owns
// every HIP call: it admits queued requests in arrival order while a slot is
// free and the request's device bytes fit (the HBM budget given at creation,
// or the device's free HBM read at admission time; reusing a cached work
// buffer of the same length, or allocating one, or evicting idle cached
// buffers of other lengths), enqueues the host-to-device copy and the whole
// search on the slot's stream, and polls slots for completion without
// blocking: a finished search's records are copied asynchronously into a
// page-locked result buffer (from a pool), and the request completes when
// that copy has.  Slots run concurrently, so requests arriving while others
// are on the GPU join the work already in flight.  The kernels take no
// decision that depends on what else is running, so each result equals the
// same series searched alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "capi_internal.hpp"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    uint64_t tag = 0;
    int64_t nsamp = 0;
    float *host = nullptr;  // pinned staging (owned by the server's pool)
    clk::time_point t_submit;
};

// Page-locked record buffer of a finished request (from the server's pool).
struct Pinned {
    fdas_cand *p = nullptr;
    int64_t cap = 0;
};

struct Result {
    uint64_t tag = 0;
    fdas_status status = FDAS_OK;
    std::string error;
    Pinned recs;     // the first n records
    int64_t n = 0;
    int64_t found = 0;
    double latency = 0.0;
};

struct Buffers {
    fdas::Workspace ws;
    float *series = nullptr;  // device copy of the request's series
    int64_t bytes = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;    // search and count copy finished
    hipEvent_t copied = nullptr;  // records copied into `out`
    bool busy = false;
    bool copying = false;
    Request req;
    Buffers *buf = nullptr;
    Pinned out;
    int64_t n = 0, found = 0;
    bool lost = false;
};

}  // namespace

struct fdas_server_s {
    fdas_plan_s *core = nullptr;  // options, thresholds, bank; no work buffers
    int64_t max_nsamp = 0;
    int64_t budget = 0;   // fixed budget; 0 = the device's free HBM at admission time
    int64_t reserve = 0;  // free HBM left untouched in that mode
    int64_t used = 0;     // device bytes held by work buffers
    std::vector<Slot> slots;
    std::multimap<int64_t, Buffers *> idle;  // cached buffers by length

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::deque<Result> done;
    std::map<int64_t, std::vector<float *>> pinned;  // free staging by length
    std::vector<Pinned> result_pool;                  // free page-locked record buffers
    int64_t outstanding = 0;
    bool stop = false;
    std::thread thread;
};

namespace fdas {

static int64_t buffer_bytes(const fdas_plan_s *core, int64_t nsamp) {
    const Geometry g = make_geometry(nsamp, core->S, core->h, core->W, cols_per_bin(core));
    return series_bytes(g, core->S, core->nz) + nsamp * 4 + candidate_bytes(core, g);
}

static void free_buffers(Buffers *b) {
    if (!b) return;
    destroy_workspace(b->ws);
    if (b->series) (void)hipFree(b->series);
    delete b;
}

// A free page-locked record buffer of at least n records (scheduler thread).
static bool take_result_buffer(fdas_server_s *sv, int64_t n, Pinned *out) {
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (size_t i = 0; i < sv->result_pool.size(); ++i) {
            if (sv->result_pool[i].cap >= n) {
                *out = sv->result_pool[i];
                sv->result_pool.erase(sv->result_pool.begin() + std::ptrdiff_t(i));
                return true;
            }
        }
    }
    int64_t cap = 4096;
    while (cap < n) cap *= 2;
    Pinned b;
    if (hipHostMalloc(reinterpret_cast<void **>(&b.p), size_t(cap) * sizeof(fdas_cand), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    b.cap = cap;
    *out = b;
    return true;
}

// Whether `need` more device bytes may be allocated now.
static bool fits(fdas_server_s *sv, int64_t need) {
    if (sv->budget > 0) return sv->used + need <= sv->budget;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
    return int64_t(fr) - sv->reserve >= need;
}

// Scheduler thread: admission, launch, completion.
static void scheduler(fdas_server_s *sv) {
    (void)hipSetDevice(sv->core->device);
    for (;;) {
        bool progressed = false;
        // ---- completions: search done -> records copied -> result
        for (Slot &sl : sv->slots) {
            if (!sl.busy) continue;
            Result res;
            res.tag = sl.req.tag;
            bool finished = false;
            if (!sl.copying) {
                const hipError_t q = hipEventQuery(sl.done);
                if (q == hipErrorNotReady) continue;
                Workspace &ws = sl.buf->ws;
                if (q != hipSuccess) {
                    res.status = FDAS_E_DEVICE;
                    res.error = std::string("request failed: ") + hipGetErrorString(q);
                    finished = true;
                } else {
                    sl.found = ws.h_count[0];
                    sl.lost = ws.h_count[2] != 0;
                    sl.n = std::min<int64_t>(sl.found, sv->core->cand_cap);
                    hipError_t e = hipSuccess;
                    if (sl.n > 0) {
                        if (!take_result_buffer(sv, sl.n, &sl.out)) {
                            res.status = FDAS_E_NOMEM;
                            res.error = "page-locked result buffer allocation failed";
                            finished = true;
                        } else {
                            e = hipMemcpyAsync(sl.out.p, ws.final, size_t(sl.n) * sizeof(fdas_cand),
                                               hipMemcpyDeviceToHost, sl.stream);
                        }
                    }
                    if (!finished) {
                        if (e == hipSuccess) e = hipEventRecord(sl.copied, sl.stream);
                        if (e != hipSuccess) {
                            res.status = FDAS_E_DEVICE;
                            res.error = std::string("copy candidates: ") + hipGetErrorString(e);
                            finished = true;
                        } else {
                            sl.copying = true;
                            progressed = true;
                            continue;
                        }
                    }
                }
            } else {
                const hipError_t q = hipEventQuery(sl.copied);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) {
                    res.status = FDAS_E_DEVICE;
                    res.error = std::string("copy candidates: ") + hipGetErrorString(q);
                } else {
                    res.recs = sl.out;
                    sl.out = Pinned{};
                    res.n = sl.n;
                    res.found = sl.found;
                    if (sl.lost) {
                        res.status = FDAS_E_OVERFLOW;
                        res.error = "harmonic-sum cell list capacity exceeded: candidates incomplete "
                                    "(raise cand_capacity)";
                    } else if (sl.found > int64_t(sv->core->cand_cap)) {
                        res.status = FDAS_E_OVERFLOW;
                        res.error = "candidate capacity exceeded";
                    }
                }
                finished = true;
            }
            if (!finished) continue;
            res.latency = std::chrono::duration<double>(clk::now() - sl.req.t_submit).count();
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sl.out.p) sv->result_pool.push_back(sl.out);  // an error left it unused
            sl.out = Pinned{};
            sv->pinned[sl.req.nsamp].push_back(sl.req.host);
            sv->idle.emplace(sl.req.nsamp, sl.buf);
            sl.buf = nullptr;
            sl.busy = false;
            sl.copying = false;
            sv->done.push_back(std::move(res));
            sv->cv_done.notify_all();
            progressed = true;
        }
        // ---- admission, in arrival order
        for (;;) {
            Slot *free_slot = nullptr;
            for (Slot &sl : sv->slots)
                if (!sl.busy) {
                    free_slot = &sl;
                    break;
                }
            Request req;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                if (!free_slot || sv->pending.empty()) break;
                req = sv->pending.front();
            }
            Buffers *buf = nullptr;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                auto it = sv->idle.find(req.nsamp);
                if (it != sv->idle.end()) {
                    buf = it->second;
                    sv->idle.erase(it);
                }
            }
            if (!buf) {
                const int64_t need = buffer_bytes(sv->core, req.nsamp);
                // evict idle buffers of other lengths until the request fits
                for (;;) {
                    if (fits(sv, need)) break;
                    Buffers *victim = nullptr;
                    {
                        std::lock_guard<std::mutex> lk(sv->mu);
                        if (sv->idle.empty()) break;
                        auto it = sv->idle.begin();
                        victim = it->second;
                        sv->idle.erase(it);
                    }
                    sv->used -= victim->bytes;
                    free_buffers(victim);
                }
                if (!fits(sv, need)) break;  // wait for a running request to finish
                buf = new Buffers;
                buf->bytes = need;
                fdas_status s = alloc_workspace(sv->core, buf->ws, req.nsamp);
                hipError_t e = hipSuccess;
                if (s == FDAS_OK) e = hipMalloc(reinterpret_cast<void **>(&buf->series), size_t(req.nsamp) * 4);
                if (s != FDAS_OK || e != hipSuccess) {
                    (void)hipGetLastError();
                    free_buffers(buf);
                    buf = nullptr;
                    // fail this request rather than block the queue
                    Result res;
                    res.tag = req.tag;
                    res.status = FDAS_E_NOMEM;
                    res.error = "device allocation for request failed";
                    std::lock_guard<std::mutex> lk(sv->mu);
                    sv->pending.pop_front();
                    sv->pinned[req.nsamp].push_back(req.host);
                    sv->done.push_back(std::move(res));
                    sv->cv_done.notify_all();
                    progressed = true;
                    continue;
                }
                sv->used += need;
            }
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->pending.pop_front();
            }
            free_slot->req = req;
            free_slot->buf = buf;
            free_slot->busy = true;
            hipStream_t st = free_slot->stream;
            hipError_t e = hipMemcpyAsync(buf->series, req.host, size_t(req.nsamp) * 4, hipMemcpyHostToDevice, st);
            fdas_status s = FDAS_OK;
            if (e == hipSuccess) {
                const Geometry g = make_geometry(req.nsamp, sv->core->S, sv->core->h, sv->core->W,
                                                 cols_per_bin(sv->core));
                s = enqueue_search(sv->core, buf->ws, g, FDAS_IN_SERIES_F32, buf->series, buf->ws.plane,
                                   buf->ws.cands, buf->ws.count, st);
                if (s == FDAS_OK) e = hipMemcpyAsync(buf->ws.h_count, buf->ws.count, 24, hipMemcpyDeviceToHost, st);
            }
            if (e == hipSuccess && s == FDAS_OK) e = hipEventRecord(free_slot->done, st);
            if (e != hipSuccess || s != FDAS_OK) {
                // launch failed: report it now and free the slot
                Result res;
                res.tag = req.tag;
                res.status = s != FDAS_OK ? s : FDAS_E_DEVICE;
                res.error = s != FDAS_OK ? g_last_error : std::string(hipGetErrorString(e));
                (void)hipStreamSynchronize(st);
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->pinned[req.nsamp].push_back(req.host);
                sv->idle.emplace(req.nsamp, buf);
                free_slot->buf = nullptr;
                free_slot->busy = false;
                sv->done.push_back(std::move(res));
                sv->cv_done.notify_all();
            }
            progressed = true;
        }
        // ---- idle wait
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->stop) {
            bool any_busy = false;
            for (Slot &sl : sv->slots) any_busy |= sl.busy;
            if (!any_busy) break;
        }
        if (!progressed) {
            bool any_busy = false;
            for (Slot &sl : sv->slots) any_busy |= sl.busy;
            if (any_busy)
                sv->cv_work.wait_for(lk, std::chrono::microseconds(100));
            else
                sv->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

}  // namespace fdas

using namespace fdas;

extern "C" {

fdas_status fdas_server_create(const fdas_bank *bank, int32_t seg, const fdas_opts *opts, int64_t max_nsamp,
                               size_t hbm_budget, int32_t max_slots, fdas_server **out) {
    if (!out || !bank || max_slots < 1 || max_slots > 64) {
        set_error("bad server arguments (max_slots in [1, 64])");
        return FDAS_E_INVAL;
    }
    *out = nullptr;
    fdas_plan_s *core = nullptr;
    fdas_status s = make_plan_core(bank, max_nsamp, seg, opts, &core);
    if (s != FDAS_OK) return s;
    auto *sv = new fdas_server_s;
    sv->core = core;
    sv->max_nsamp = max_nsamp;
    sv->budget = int64_t(hbm_budget);
    {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = tot = 0;
        sv->reserve = (int64_t(512) << 20) + int64_t(tot / 100);
        const int64_t room = hbm_budget ? sv->budget : int64_t(fr) - sv->reserve;
        if (room < buffer_bytes(core, max_nsamp)) {
            fdas_plan_destroy(core);
            delete sv;
            set_error(hbm_budget ? "HBM budget smaller than one request of max_nsamp"
                                 : "free HBM smaller than one request of max_nsamp");
            return FDAS_E_NOMEM;
        }
    }
    sv->slots.resize(size_t(max_slots));
    for (Slot &sl : sv->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (Slot &x : sv->slots) {
                if (x.stream) (void)hipStreamDestroy(x.stream);
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.copied) (void)hipEventDestroy(x.copied);
            }
            fdas_plan_destroy(core);
            delete sv;
            set_error(std::string("server streams: ") + hipGetErrorString(e));
            return FDAS_E_DEVICE;
        }
    }
    sv->thread = std::thread(scheduler, sv);
    *out = sv;
    return FDAS_OK;
}

fdas_status fdas_submit(fdas_server *sv, const float *series_host, int64_t nsamp, uint64_t tag) {
    if (!sv || !series_host) {
        set_error("bad submit arguments");
        return FDAS_E_INVAL;
    }
    fdas_status s = check_nsamp(nsamp, sv->core->S, sv->core->h);
    if (s != FDAS_OK) return s;
    if (nsamp > sv->max_nsamp || nsamp / 2 < int64_t(sv->core->W)) {
        set_error("series length outside [2 W, max_nsamp]");
        return FDAS_E_INVAL;
    }
    float *host = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->pending.size() >= 65536) {
            set_error("server queue full");
            return FDAS_E_BUSY;
        }
        auto &pool = sv->pinned[nsamp];
        if (!pool.empty()) {
            host = pool.back();
            pool.pop_back();
        }
    }
    if (!host) {
        if (hipHostMalloc(reinterpret_cast<void **>(&host), size_t(nsamp) * 4, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("pinned host allocation failed");
            return FDAS_E_NOMEM;
        }
    }
    std::memcpy(host, series_host, size_t(nsamp) * 4);
    Request r;
    r.tag = tag;
    r.nsamp = nsamp;
    r.host = host;
    r.t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->pending.push_back(r);
        ++sv->outstanding;
    }
    sv->cv_work.notify_all();
    return FDAS_OK;
}

fdas_status fdas_poll(fdas_server *sv, uint64_t *tag, fdas_cand *cands, int64_t cap, int64_t *ncands,
                      double *latency_s, int32_t timeout_ms) {
    if (!sv || cap < 0 || (cap > 0 && !cands)) {
        set_error("bad poll arguments");
        return FDAS_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return !sv->done.empty(); };
    if (timeout_ms < 0)
        sv->cv_done.wait(lk, ready);
    else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        set_error("no request completed within the timeout");
        return FDAS_E_TIMEOUT;
    }
    Result res = std::move(sv->done.front());
    sv->done.pop_front();
    --sv->outstanding;
    lk.unlock();
    if (tag) *tag = res.tag;
    if (latency_s) *latency_s = res.latency;
    const int64_t n = std::min<int64_t>(res.n, cap);
    if (n > 0) std::memcpy(cands, res.recs.p, size_t(n) * sizeof(fdas_cand));
    if (res.recs.p) {
        std::lock_guard<std::mutex> lk2(sv->mu);
        sv->result_pool.push_back(res.recs);
    }
    if (ncands) *ncands = res.status == FDAS_OK || res.status == FDAS_E_OVERFLOW ? res.found : 0;
    if (res.status != FDAS_OK) {
        set_error(res.error);
        return res.status;
    }
    if (res.found > cap) {
        set_error("candidate capacity exceeded");
        return FDAS_E_OVERFLOW;
    }
    return FDAS_OK;
}

int64_t fdas_server_outstanding(const fdas_server *sv) {
    if (!sv) return 0;
    std::lock_guard<std::mutex> lk(const_cast<fdas_server *>(sv)->mu);
    return sv->outstanding;
}

void fdas_server_destroy(fdas_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        for (Request &r : sv->pending) sv->pinned[r.nsamp].push_back(r.host);
        sv->pending.clear();
    }
    sv->cv_work.notify_all();
    if (sv->thread.joinable()) sv->thread.join();
    for (Slot &sl : sv->slots) {
        if (sl.buf) free_buffers(sl.buf);
        if (sl.out.p) (void)hipHostFree(sl.out.p);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.copied) (void)hipEventDestroy(sl.copied);
    }
    for (Pinned &b : sv->result_pool) (void)hipHostFree(b.p);
    for (Result &r : sv->done)
        if (r.recs.p) (void)hipHostFree(r.recs.p);
    for (auto &kv : sv->idle) free_buffers(kv.second);
    for (auto &kv : sv->pinned)
        for (float *p : kv.second) (void)hipHostFree(p);
    fdas_plan_destroy(sv->core);
    delete sv;
}

}  // extern "C"
