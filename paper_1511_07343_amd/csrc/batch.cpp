// fdas_search_batch: many series through the hot path, in one of two forms.
//
// Two streams (the default, and every plan the persistent form does not
// cover): consecutive trials on two streams and two work buffers, each
// slot's per-trial launch sequence captured once per series length in a HIP
// graph that reads the workspace's own input buffer (a trial is a
// device-to-device copy into that buffer followed by a graph launch).  One
// trial's memory-bound harmonic sums overlap the next trial's ALU-bound
// correlation, each kernel at its own occupancy.
//
// Persistent (opts.batch_launch = FDAS_BATCH_PERSISTENT; segment lengths 4096
// and 8192 of the FFT correlator, no half-bin plane): up to 64 trials of
// mixed lengths go through ONE launch of a persistent kernel.  Per trial, the
// real DFT and block medians run first (small launches); then the persistent
// workgroups take tiles from a device work queue (the global tile order
// built here): segment DFTs, correlation tiles (segment x template block),
// harmonic-sum screen tiles, exact-sum and neighbour-test tiles.  A
// per-trial, per-stage completion counter releases the next stage's tiles of
// that trial, and the stages of consecutive trials are interleaved, so one
// trial's harmonic sums run beside the next trial's correlation.  Planes,
// codes and harmonic-sum lists live in a ring of kBatchSlots slots: trial
// t's correlation waits until trial t - kBatchSlots has finished its
// neighbour test.  The upload of the order, the clears, the per-trial front
// end, the persistent launch and the copy-back of the counts are captured in
// one HIP graph per call; candidate sorting and the copies to the host
// follow per trial.  Every tile runs at the correlation tiles' occupancy
// (two workgroups per CU), which slows the memory-bound harmonic-sum tiles:
// on MI355X this form reaches about 0.6 of the two-stream rate.
#include <algorithm>
#include <string>
#include <vector>

#include "capi_internal.hpp"

namespace fdas {

constexpr int kBatchSlots = 4;

struct PBatch {
    int trials = 0;      // per-trial buffers are allocated for this many trials
    int64_t nsamp = 0;   // ... of at most this length
    int64_t x_stride = 0, med_stride = 0, seg_stride = 0;  // elements per trial
    float2 *Z = nullptr, *work = nullptr;  // front-end scratch
    float2 *X = nullptr;
    double *med = nullptr;
    float2 *seg = nullptr;
    DevCand *cands = nullptr;
    uint32_t *cnt = nullptr;  // 8 words per trial
    std::array<float *, kBatchSlots> plane{};
    std::array<uint8_t *, kBatchSlots> codes{};
    std::array<void *, kBatchSlots> hits{};
    uint32_t *ctl = nullptr;
    BatchTrial *d_trials = nullptr;
    uint32_t *d_tiles = nullptr;
    size_t tiles_cap = 0;
    BatchTrial *h_trials = nullptr;  // page-locked staging of the upload
    uint32_t *h_tiles = nullptr;
    uint32_t *h_cnt = nullptr;       // page-locked copy-back: 8 words per trial, then the control head
    void *sort = nullptr;
    fdas_cand *final = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    int workgroups = 0;
};

static void free_pbatch_buffers(PBatch *pb) {
    for (void *q : {(void *)pb->Z, (void *)pb->work, (void *)pb->X, (void *)pb->med, (void *)pb->seg,
                    (void *)pb->cands, (void *)pb->cnt, (void *)pb->ctl, (void *)pb->d_trials, (void *)pb->d_tiles,
                    pb->sort, (void *)pb->final})
        if (q) (void)hipFree(q);
    for (int i = 0; i < kBatchSlots; ++i) {
        if (pb->plane[size_t(i)]) (void)hipFree(pb->plane[size_t(i)]);
        if (pb->codes[size_t(i)]) (void)hipFree(pb->codes[size_t(i)]);
        if (pb->hits[size_t(i)]) (void)hipFree(pb->hits[size_t(i)]);
    }
    for (void *q : {(void *)pb->h_trials, (void *)pb->h_tiles, (void *)pb->h_cnt})
        if (q) (void)hipHostFree(q);
    pb->Z = pb->work = pb->X = pb->seg = nullptr;
    pb->med = nullptr;
    pb->cands = nullptr;
    pb->cnt = pb->ctl = pb->d_tiles = pb->h_tiles = pb->h_cnt = nullptr;
    pb->d_trials = pb->h_trials = nullptr;
    pb->sort = nullptr;
    pb->final = nullptr;
    pb->plane = {};
    pb->codes = {};
    pb->hits = {};
    pb->trials = 0;
    pb->nsamp = 0;
    pb->tiles_cap = 0;
}

void destroy_pbatch(PBatch *pb) {
    if (!pb) return;
    if (pb->st) (void)hipStreamSynchronize(pb->st);
    free_pbatch_buffers(pb);
    if (pb->st) (void)hipStreamDestroy(pb->st);
    if (pb->ev) (void)hipEventDestroy(pb->ev);
    delete pb;
}

// Whether the persistent launch serves this plan.
static bool persistent_ok(const fdas_plan_s *p) {
    return p->opts.batch_launch == FDAS_BATCH_PERSISTENT && !p->td && p->corr == FDAS_CORR_FFT_F32 && !p->opts.interbin && (p->log2s == 12 || p->log2s == 13) &&
           p->nz <= 65535 && p->nsamp / 2 >= 32;
}

// Buffers for `trials` trials of at most the plan's length, the slot ring
// and a tile table of `tiles` entries (grown, never shrunk).
static fdas_status ensure_pbatch(fdas_plan_s *p, int trials, size_t tiles) {
    if (!p->pbatch) p->pbatch = new PBatch();
    PBatch *pb = p->pbatch;
    hipError_t e;
    if (!pb->st) {
        e = hipStreamCreateWithFlags(&pb->st, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(p, e, "batch stream");
        e = hipEventCreateWithFlags(&pb->ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(p, e, "batch event");
        int per_cu = 0;
        e = batch_persistent_workgroups(p->log2s, p->opts.nharm_max, &per_cu);
        if (e != hipSuccess || per_cu <= 0) {
            set_error("persistent batch kernel does not fit the device");
            return FDAS_E_DEVICE;
        }
        pb->workgroups = per_cu * p->num_cu;
    }
    auto fail_nomem = [&](const char *what) {
        (void)hipGetLastError();
        free_pbatch_buffers(pb);
        set_error(std::string("batch allocation: ") + what);
        return FDAS_E_NOMEM;
    };
#define PB_ALLOC(ptr, bytes)                                                           do {                                                                                   if (hipMalloc(reinterpret_cast<void **>(&(ptr)), size_t(bytes)) != hipSuccess)             return fail_nomem(#ptr);                                                   } while (0)
    if (pb->trials < trials || pb->nsamp != p->nsamp) {
        free_pbatch_buffers(pb);
        const Geometry g = make_geometry(p->nsamp, p->S, p->h, p->W, 1);
        pb->x_stride = g.nb;
        pb->med_stride = g.nblk;
        pb->seg_stride = g.nseg * int64_t(p->S);
        PB_ALLOC(pb->Z, g.nb * 8);
        PB_ALLOC(pb->work, g.nb * 8);
        PB_ALLOC(pb->X, int64_t(trials) * pb->x_stride * 8);
        PB_ALLOC(pb->med, int64_t(trials) * pb->med_stride * 8);
        PB_ALLOC(pb->seg, int64_t(trials) * pb->seg_stride * 8);
        PB_ALLOC(pb->cands, int64_t(trials) * int64_t(p->cand_cap) * int64_t(sizeof(DevCand)));
        PB_ALLOC(pb->cnt, int64_t(trials) * 8 * 4);
        for (int i = 0; i < kBatchSlots; ++i) {
            PB_ALLOC(pb->plane[size_t(i)], int64_t(p->nz) * g.nb * 4);
            PB_ALLOC(pb->codes[size_t(i)], int64_t(p->nz) * (g.nb / 2));
            PB_ALLOC(pb->hits[size_t(i)], harmsum_scratch_bytes(p->nz, g.nb, p->hit_cap, p->group_cap));
        }
        PB_ALLOC(pb->ctl, (kBatchCtlHead + BST_N * kBatchMaxTrials) * 4);
        PB_ALLOC(pb->d_trials, kBatchMaxTrials * sizeof(BatchTrial));
        PB_ALLOC(pb->sort, cand_sort_scratch_bytes(p->cand_cap));
        PB_ALLOC(pb->final, int64_t(p->cand_cap) * int64_t(sizeof(fdas_cand)));
        if (hipHostMalloc(reinterpret_cast<void **>(&pb->h_trials), kBatchMaxTrials * sizeof(BatchTrial),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&pb->h_cnt), (kBatchMaxTrials * 8 + kBatchCtlHead) * 4,
                          hipHostMallocDefault) != hipSuccess)
            return fail_nomem("page-locked staging");
        pb->trials = trials;
        pb->nsamp = p->nsamp;
    }
    if (pb->tiles_cap < tiles) {
        if (pb->d_tiles) (void)hipFree(pb->d_tiles);
        if (pb->h_tiles) (void)hipHostFree(pb->h_tiles);
        pb->d_tiles = pb->h_tiles = nullptr;
        pb->tiles_cap = 0;
        PB_ALLOC(pb->d_tiles, tiles * 4);
        if (hipHostMalloc(reinterpret_cast<void **>(&pb->h_tiles), tiles * 4, hipHostMallocDefault) != hipSuccess)
            return fail_nomem("page-locked tile order");
        pb->tiles_cap = tiles;
    }
#undef PB_ALLOC
    return FDAS_OK;
}

// Tiles of each stage of a trial of nsamp samples.
static void stage_tiles(const fdas_plan_s *p, int64_t nsamp, uint32_t (&nt)[BST_N], int64_t *nb, int64_t *nseg) {
    const Geometry g = make_geometry(nsamp, p->S, p->h, p->W, 1);
    const int64_t nzb = (p->nz + p->tpb - 1) / p->tpb;
    nt[BST_SEG] = uint32_t(g.nseg);
    nt[BST_CORR] = uint32_t(g.nseg * nzb);
    nt[BST_SCREEN] = batch_screen_tiles(g.nb, p->nz);
    nt[BST_EXACT] = kBatchExactTiles;
    nt[BST_PEAK] = kBatchPeakTiles;
    *nb = g.nb;
    *nseg = g.nseg;
}

// The global tile order of m trials (see the file comment).  Step u holds
// the segment DFTs of trial u + 1, the correlation of trial u, the screen of
// trial u - 1, the exact sums of trial u - 2 and the neighbour test of trial
// u - 3: every tile's dependencies were issued at least one step earlier,
// except the correlation's on its segment DFTs (issued at the head of the
// previous step) and the first steps'.  The correlation's first 2 G tiles
// (G workgroups) lead its step, so that the previous step's tiles have
// drained before the dependent stages' tiles are taken; the screen tiles are
// then spread evenly over the rest of the correlation.
static size_t build_order(const std::vector<std::array<uint32_t, BST_N>> &nt, int workgroups, uint32_t *out) {
    const int m = int(nt.size());
    size_t k = 0;
    auto emit = [&](uint32_t stage, int trial, uint32_t first, uint32_t count) {
        for (uint32_t i = 0; i < count; ++i) {
            if (out) out[k] = batch_tile(stage, uint32_t(trial), first + i);
            ++k;
        }
    };
    auto valid = [&](int t) { return t >= 0 && t < m; };
    for (int u = -1; u < m + 3; ++u) {
        if (valid(u + 1)) emit(BST_SEG, u + 1, 0, nt[size_t(u + 1)][BST_SEG]);
        const uint32_t ncorr = valid(u) ? nt[size_t(u)][BST_CORR] : 0;
        const uint32_t head = std::min<uint32_t>(ncorr, uint32_t(2 * workgroups));
        if (head) emit(BST_CORR, u, 0, head);
        if (valid(u - 2)) emit(BST_EXACT, u - 2, 0, nt[size_t(u - 2)][BST_EXACT]);
        if (valid(u - 3)) emit(BST_PEAK, u - 3, 0, nt[size_t(u - 3)][BST_PEAK]);
        const uint32_t rest = ncorr - head;
        const uint32_t nscr = valid(u - 1) ? nt[size_t(u - 1)][BST_SCREEN] : 0;
        const uint32_t chunks = std::max<uint32_t>(1, rest / 32);
        uint32_t ci = head, si = 0;
        for (uint32_t c = 0; c < chunks; ++c) {
            const uint32_t ce = head + uint32_t(uint64_t(rest) * (c + 1) / chunks);
            const uint32_t se = uint32_t(uint64_t(nscr) * (c + 1) / chunks);
            if (ce > ci) emit(BST_CORR, u, ci, ce - ci);
            if (se > si) emit(BST_SCREEN, u - 1, si, se - si);
            ci = ce;
            si = se;
        }
    }
    return k;
}

// One persistent launch for trials [i0, i0 + m) of the batch.
static fdas_status run_persistent_chunk(fdas_plan_s *p, int i0, int m, const float *const *series_dev,
                                        const int64_t *nsamp, fdas_cand *cands_host, const int64_t *cap,
                                        const int64_t *offset, int64_t *ncands, bool *overflow) {
    const size_t mm = static_cast<size_t>(m);
    std::vector<std::array<uint32_t, BST_N>> nt(mm);
    std::vector<int64_t> nbs(mm), nsegs(mm);
    for (int i = 0; i < m; ++i) {
        uint32_t t[BST_N];
        stage_tiles(p, nsamp[i0 + i], t, &nbs[size_t(i)], &nsegs[size_t(i)]);
        for (int s = 0; s < BST_N; ++s) {
            if (t[s] >= kBatchMaxStageTiles) {
                set_error("batch trial has too many tiles");
                return FDAS_E_INVAL;
            }
            nt[size_t(i)][size_t(s)] = t[s];
        }
    }
    const int wg_guess = p->pbatch ? p->pbatch->workgroups : 0;
    const size_t ntiles = build_order(nt, std::max(wg_guess, 1), nullptr);
    fdas_status s = ensure_pbatch(p, std::max(m, p->pbatch ? p->pbatch->trials : 0), ntiles);
    if (s != FDAS_OK) return s;
    PBatch *pb = p->pbatch;
    const size_t nt2 = build_order(nt, pb->workgroups, pb->h_tiles);
    if (nt2 != ntiles || ntiles > 0xffffffffu) {
        set_error("batch tile order");
        return FDAS_E_DEVICE;
    }
    for (int i = 0; i < m; ++i) {
        BatchTrial &d = pb->h_trials[i];
        const int sl = i % kBatchSlots;
        d.X = pb->X + int64_t(i) * pb->x_stride;
        d.med = pb->med + int64_t(i) * pb->med_stride;
        d.seg = pb->seg + int64_t(i) * pb->seg_stride;
        d.plane = pb->plane[size_t(sl)];
        d.codes = pb->codes[size_t(sl)];
        d.hits = pb->hits[size_t(sl)];
        d.cnt = pb->cnt + int64_t(i) * 8;
        d.cands = pb->cands + int64_t(i) * int64_t(p->cand_cap);
        d.nb = nbs[size_t(i)];
        d.nseg = nsegs[size_t(i)];
        for (int st = 0; st < BST_N; ++st) d.ntile[st] = nt[size_t(i)][size_t(st)];
        d.pad = 0;
    }
    // capture: upload, clears, front end, the persistent launch, counts back
    hipStream_t st = pb->st;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(p, e, "begin capture");
    auto enqueue = [&]() -> hipError_t {
        hipError_t r;
        if ((r = hipMemcpyAsync(pb->d_trials, pb->h_trials, size_t(m) * sizeof(BatchTrial), hipMemcpyHostToDevice,
                                st)) != hipSuccess)
            return r;
        if ((r = hipMemcpyAsync(pb->d_tiles, pb->h_tiles, ntiles * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
            return r;
        if ((r = launch_zero_u32(pb->ctl, kBatchCtlHead + BST_N * m, st)) != hipSuccess) return r;
        if ((r = launch_zero_u32(pb->cnt, 8 * m, st)) != hipSuccess) return r;
        for (int i = 0; i < m; ++i) {
            if ((r = launch_r2c_packed(series_dev[i0 + i], nsamp[i0 + i], pb->Z, pb->work, st)) != hipSuccess)
                return r;
            if ((r = launch_unpack_median(pb->Z, nsamp[i0 + i], const_cast<float2 *>(pb->h_trials[i].X),
                                          const_cast<double *>(pb->h_trials[i].med), p->W, st)) != hipSuccess)
                return r;
        }
        if ((r = launch_batch_persistent(p->log2s, p->opts.nharm_max, pb->d_trials, m, pb->d_tiles,
                                         uint32_t(ntiles), pb->ctl, kBatchSlots, p->d_bank, p->nz, p->tpb, p->h,
                                         p->W, p->izc, p->code_inv, p->thr_f, p->code_thr, p->hit_cap, p->group_cap,
                                         p->cand_cap, pb->workgroups, st)) != hipSuccess)
            return r;
        if ((r = hipMemcpyAsync(pb->h_cnt, pb->cnt, size_t(m) * 8 * 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
            return r;
        return hipMemcpyAsync(pb->h_cnt + kBatchMaxTrials * 8, pb->ctl, kBatchCtlHead * 4, hipMemcpyDeviceToHost,
                              st);
    };
    const hipError_t eq = enqueue();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (eq != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(p, eq, "batch enqueue");
    }
    if (e != hipSuccess) return hip_fail(p, e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(p, e, "graph instantiate");
    e = hipGraphLaunch(exec, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
    if (e != hipSuccess) return hip_fail(p, e, "persistent batch");
    const uint32_t *head = pb->h_cnt + kBatchMaxTrials * 8;
    if (head[1] != 0) {
        if (head[1] == 2u) {
            set_error("persistent batch: malformed tile order");
        } else {
            static const char *names[BST_N] = {"segment DFT", "correlation", "screen", "exact sums", "neighbour test"};
            set_error(std::string("persistent batch: a dependency wait ran out (") +
                      (head[2] < BST_N ? names[head[2]] : "?") + " of trial " + std::to_string(i0 + int(head[3])) +
                      ": " + std::to_string(head[4]) + " of " + std::to_string(head[5]) + " tiles done)");
        }
        p->broken = true;
        return FDAS_E_DEVICE;
    }
    // sort each trial's records and copy them out
    for (int i = 0; i < m; ++i) {
        const uint32_t found = pb->h_cnt[i * 8 + 0];
        const bool lost = pb->h_cnt[i * 8 + 2] != 0;
        const int j = i0 + i;
        const int64_t n = std::min<int64_t>(std::min<int64_t>(found, p->cand_cap), cap[j]);
        ncands[j] = found;
        if (n > 0) {
            e = launch_finish_candidates(pb->h_trials[i].cands, pb->h_trials[i].cnt, p->cand_cap, pb->sort, p->nz,
                                         nbs[size_t(i)], 1, p->zmax, p->dz, pb->final, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cands_host + offset[j], pb->final, size_t(n) * sizeof(fdas_cand),
                                   hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return hip_fail(p, e, "batch candidates");
        }
        if (lost || int64_t(found) > cap[j] || found > p->cand_cap) *overflow = true;
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(p, e, "batch candidates");
    return FDAS_OK;
}

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
    if (persistent_ok(plan)) {
        std::vector<int64_t> off(size_t(n) + 1, 0);
        for (int32_t i = 0; i < n; ++i) off[size_t(i) + 1] = off[size_t(i)] + cap[i];
        hipStream_t user = static_cast<hipStream_t>(hip_stream);
        if (!plan->pbatch || !plan->pbatch->st) {
            fdas_status s0 = ensure_pbatch(plan, 0, 0);
            if (s0 != FDAS_OK) return s0;
        }
        // the batch starts after what the caller's stream holds
        hipError_t e = hipEventRecord(plan->pbatch->ev, user);
        if (e == hipSuccess) e = hipStreamWaitEvent(plan->pbatch->st, plan->pbatch->ev, 0);
        if (e != hipSuccess) return hip_fail(plan, e, "stream order");
        bool overflow = false;
        for (int32_t i0 = 0; i0 < n; i0 += kBatchMaxTrials) {
            const int m = std::min<int>(kBatchMaxTrials, n - i0);
            fdas_status s = run_persistent_chunk(plan, i0, m, series_dev, nsamp, cands_host, cap, off.data(), ncands,
                                                 &overflow);
            if (s != FDAS_OK) return s;
        }
        if (overflow) {
            set_error("candidate capacity exceeded in a batch trial");
            return FDAS_E_OVERFLOW;
        }
        return FDAS_OK;
    }
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
