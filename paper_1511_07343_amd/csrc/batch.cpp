// fdas_search_batch: many series through the hot path with consecutive trials
// on two streams and two work buffers, so that one trial's memory-bound
// harmonic sum runs beside the next trial's ALU-bound correlation.  Each
// slot's per-trial launch sequence is captured once per series length in a
// HIP graph that reads the workspace's own input buffer; a trial is a
// device-to-device copy into that buffer followed by a graph launch.
#include <algorithm>
#include <string>

#include "capi_internal.hpp"

namespace fdas {

// Workspace of batch slot i (0 or 1): plan->ws[1 + i], never the buffers of
// fdas_search.
static fdas::Workspace &slot_ws(fdas_plan_s *p, int i) { return p->ws[size_t(1 + i)]; }

static fdas_status ensure_batch_resources(fdas_plan_s *p) {
    for (int i = 0; i < 2; ++i) {
        if (!slot_ws(p, i).nsamp) {
            fdas_status s = alloc_workspace(p, slot_ws(p, i), p->nsamp);
            if (s != FDAS_OK) return s;
        }
        if (!slot_ws(p, i).series) {
            hipError_t e = hipMalloc(reinterpret_cast<void **>(&slot_ws(p, i).series), size_t(p->nsamp) * 4);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipMalloc batch input buffer");
                return FDAS_E_NOMEM;
            }
        }
        if (!p->aux[i]) {
            hipError_t e = hipStreamCreateWithFlags(&p->aux[i], hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(p, e, "stream create");
        }
    }
    for (hipEvent_t &ev : p->events) {
        if (!ev) {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(p, e, "event create");
        }
    }
    return FDAS_OK;
}

// The captured launch sequence of one trial of length nsamp on slot i.
static fdas_status slot_graph(fdas_plan_s *p, int i, int64_t nsamp, hipGraphExec_t *out) {
    auto it = p->graphs[size_t(i)].find(nsamp);
    if (it != p->graphs[size_t(i)].end()) {
        *out = it->second;
        return FDAS_OK;
    }
    Workspace &ws = slot_ws(p, i);
    hipStream_t st = p->aux[size_t(i)];
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(p, e, "begin capture");
    const Geometry g = make_geometry(nsamp, p->S, p->h, p->W, cols_per_bin(p));
    fdas_status s = enqueue_search(p, ws, g, FDAS_IN_SERIES_F32, ws.series, ws.plane, ws.cands, ws.count, st);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (s != FDAS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return hip_fail(p, e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(p, e, "graph instantiate");
    p->graphs[size_t(i)][nsamp] = exec;
    *out = exec;
    return FDAS_OK;
}

}  // namespace fdas

using namespace fdas;

extern "C" fdas_status fdas_search_batch(fdas_plan_t *plan, int32_t n, const float *const *series_dev,
                                         const int64_t *nsamp, fdas_cand *cands_host, const int64_t *cap,
                                         int64_t *ncands, void *hip_stream) {
    if (!plan || n < 0 || (n > 0 && (!series_dev || !nsamp || !cap || !ncands))) {
        set_error("bad batch arguments");
        return FDAS_E_INVAL;
    }
    if (plan->broken) {
        set_error("plan is unusable after a device error");
        return FDAS_E_DEVICE;
    }
    if (plan->td) {
        set_error("batches need a template (FDAS) plan");
        return FDAS_E_INVAL;
    }
    int64_t total_cap = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!series_dev[i] || cap[i] < 0) {
            set_error("bad series pointer or capacity in batch");
            return FDAS_E_INVAL;
        }
        fdas_status s = check_nsamp(nsamp[i], plan->S, plan->h);
        if (s != FDAS_OK) return s;
        if (nsamp[i] > plan->nsamp) {
            set_error("batch series longer than the plan's nsamp");
            return FDAS_E_INVAL;
        }
        total_cap += cap[i];
    }
    if (total_cap > 0 && !cands_host) {
        set_error("cands_host is NULL");
        return FDAS_E_INVAL;
    }
    if (n == 0) return FDAS_OK;
    fdas_status s = ensure_batch_resources(plan);
    if (s != FDAS_OK) return s;

    hipStream_t user = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipEventRecord(plan->events[2], user);
    if (e != hipSuccess) return hip_fail(plan, e, "event record");
    for (int i = 0; i < 2; ++i) {
        e = hipStreamWaitEvent(plan->aux[i], plan->events[2], 0);
        if (e != hipSuccess) return hip_fail(plan, e, "stream wait");
    }

    std::vector<int64_t> offset(size_t(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i) offset[size_t(i) + 1] = offset[size_t(i)] + cap[i];

    fdas_status first_err = FDAS_OK;
    bool overflow = false;
    // Finish trial j: its count is already copied (event ev[j % 2]); copy the
    // records and convert them.
    auto finish = [&](int32_t j) -> fdas_status {
        const int slot = j % 2;
        hipError_t ee = hipEventSynchronize(plan->events[slot]);
        if (ee != hipSuccess) return hip_fail(plan, ee, "batch trial");
        fdas_status r = copy_candidates(plan, slot_ws(plan, slot), cands_host + offset[size_t(j)], cap[j], &ncands[j],
                                        plan->aux[slot]);
        if (r == FDAS_E_OVERFLOW) {
            overflow = true;
            r = FDAS_OK;
        }
        return r;
    };

    for (int32_t i = 0; i < n && first_err == FDAS_OK; ++i) {
        const int slot = i % 2;
        if (i >= 2) {
            first_err = finish(i - 2);
            if (first_err != FDAS_OK) break;
        }
        Workspace &ws = slot_ws(plan, slot);
        hipGraphExec_t exec = nullptr;
        first_err = slot_graph(plan, slot, nsamp[i], &exec);
        if (first_err != FDAS_OK) break;
        e = hipMemcpyAsync(ws.series, series_dev[i], size_t(nsamp[i]) * 4, hipMemcpyDeviceToDevice, plan->aux[slot]);
        if (e == hipSuccess) e = hipGraphLaunch(exec, plan->aux[slot]);
        if (e != hipSuccess) {
            first_err = hip_fail(plan, e, "batch trial launch");
            break;
        }
        e = hipMemcpyAsync(ws.h_count, ws.count, 24, hipMemcpyDeviceToHost, plan->aux[slot]);
        if (e != hipSuccess) {
            first_err = hip_fail(plan, e, "copy candidate count");
            break;
        }
        e = hipEventRecord(plan->events[slot], plan->aux[slot]);
        if (e != hipSuccess) {
            first_err = hip_fail(plan, e, "event record");
            break;
        }
    }
    if (first_err == FDAS_OK) {
        for (int32_t j = std::max(0, n - 2); j < n && first_err == FDAS_OK; ++j) first_err = finish(j);
    }
    // order the user's stream after everything enqueued here
    for (int i = 0; i < 2; ++i) {
        if (hipEventRecord(plan->events[2 + (i & 1)], plan->aux[i]) == hipSuccess)
            (void)hipStreamWaitEvent(user, plan->events[2 + (i & 1)], 0);
    }
    if (first_err != FDAS_OK) return first_err;
    if (overflow) {
        set_error("candidate capacity exceeded in a batch trial");
        return FDAS_E_OVERFLOW;
    }
    return FDAS_OK;
}
