// C ABI of the FDAS library: template bank, plans, the per-series search, the
// batched search and test hooks.  The serving loop lives in server.cpp.
//
// Per-series steps (Sec. 4 of Dimoudi & Armour): the series is already on the
// device (step 1 is the caller's copy); real-to-complex DFT (step 2) plus the
// block-median normalisation statistics; overlapped segments (step 3, folded
// into the segment loader) and their DFTs (step 4); complex multiply by every
// template, inverse DFT and power with edge removal (steps 5-7, one fused
// kernel) into the f-fdot plane; then harmonic sums, thresholds and peaks.
#include "capi_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

namespace fdas {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
static int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

fdas_status hip_fail(fdas_plan_s *plan, hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    if (plan) plan->broken = true;
    return FDAS_E_DEVICE;
}

fdas_status validate_opts(const fdas_opts &o) {
    if (!(o.sigma > -30.0 && o.sigma < 1000.0)) {
        set_error("opts.sigma out of range");
        return FDAS_E_INVAL;
    }
    if (!(o.nharm_max == 1 || o.nharm_max == 2 || o.nharm_max == 4 || o.nharm_max == 8 || o.nharm_max == 16)) {
        set_error("opts.nharm_max must be 1, 2, 4, 8 or 16");
        return FDAS_E_INVAL;
    }
    if (o.correlator < FDAS_CORR_FFT_F32 || o.correlator > FDAS_CORR_GEMM_F16) {
        set_error("opts.correlator must be FDAS_CORR_FFT_F32, FDAS_CORR_GEMM_BF16 or FDAS_CORR_GEMM_F16");
        return FDAS_E_INVAL;
    }
    if (!is_pow2(o.median_window) || o.median_window < 32 || o.median_window > 8192) {
        set_error("opts.median_window must be a power of two in [32, 8192]");
        return FDAS_E_INVAL;
    }
    if (o.cand_capacity < 0 || o.cand_capacity > (int64_t(1) << 28)) {
        set_error("opts.cand_capacity must be in [0, 2^28] (0 = automatic)");
        return FDAS_E_INVAL;
    }
    if (o.templates_per_block < 0 || o.templates_per_block > 4096) {
        set_error("opts.templates_per_block must be in [0, 4096]");
        return FDAS_E_INVAL;
    }
    if (o.refine_levels < 0 || o.refine_levels > 20) {
        set_error("opts.refine_levels must be in [0, 20]");
        return FDAS_E_INVAL;
    }
    if (o.interbin != 0 && o.interbin != 1) {
        set_error("opts.interbin must be 0 or 1");
        return FDAS_E_INVAL;
    }
    if (o.interbin && o.correlator != FDAS_CORR_FFT_F32) {
        set_error("the half-bin plane needs the FFT correlator");
        return FDAS_E_INVAL;
    }
    if (o.batch_launch != FDAS_BATCH_PERSISTENT && o.batch_launch != FDAS_BATCH_STREAMS) {
        set_error("opts.batch_launch must be FDAS_BATCH_PERSISTENT or FDAS_BATCH_STREAMS");
        return FDAS_E_INVAL;
    }
    return FDAS_OK;
}

fdas_status check_nsamp(int64_t nsamp, int32_t seg, int32_t h) {
    if (!is_pow2(nsamp) || nsamp < 1024 || nsamp > (int64_t(1) << 26)) {
        set_error("nsamp must be a power of two in [2^10, 2^26]");
        return FDAS_E_INVAL;
    }
    (void)seg;
    (void)h;
    return FDAS_OK;
}

// Geometry of one series length under a plan's segment length.
Geometry make_geometry(int64_t nsamp, int32_t S, int32_t h, int32_t W, int cpb) {
    Geometry g;
    g.nsamp = nsamp;
    g.nb = nsamp / 2;
    g.ncol = g.nb * cpb;
    g.L = (S - 2 * h) & ~3;  // a multiple of 4: store chunks and code blocks never straddle two segments
    g.nseg = g.L > 0 ? (g.nb + g.L - 1) / g.L : 0;  // no segments without templates (time-domain search)
    g.nblk = (g.nb + W - 1) / W;
    return g;
}

// Device bytes of the per-series buffers (spectrum scratch, medians, segment
// spectra, plane and its screening codes) for a given geometry.
int64_t series_bytes(const Geometry &g, int32_t S, int32_t nz) {
    const int64_t M = g.nb;
    return 3 * M * 8 + g.nblk * 8 + g.nseg * int64_t(S) * 8 + int64_t(nz) * g.ncol * 4 + int64_t(nz) * (g.ncol / 2);
}

// Device bytes of the per-series buffers that depend on the plan's options
// (candidate buffers, harmonic-sum lists, the matrix correlator's spectrum)
// for a series of the given geometry.
int64_t candidate_bytes(const fdas_plan_s *p, const Geometry &g) {
    const uint32_t cap = p->cand_cap;
    return int64_t(cap) * int64_t(sizeof(DevCand) + sizeof(fdas_cand)) + int64_t(cand_sort_scratch_bytes(cap)) +
           int64_t(harmsum_scratch_bytes(p->nz, g.ncol, p->hit_cap, p->group_cap)) + 64 + (p->corr ? g.nb * 4 : 0);
}

// The time-domain resampling search on `st`: per trial, resample, real DFT,
// block medians, normalised powers and codes into plane row iz; then the
// harmonic sums along each row (izc < 0), peaks, candidates and their drift.
// Timing stages: 0 the trials' spectra, 4 harmonic sums to sorted
// candidates (the others stay empty).
static fdas_status enqueue_td_search(fdas_plan_s *p, const Workspace &ws, const Geometry &g, int32_t in_kind,
                                     const void *in_dev, float *plane, DevCand *dcands, uint32_t *dcount,
                                     hipStream_t st, bool timed) {
    if (in_kind != FDAS_IN_SERIES_F32) {
        set_error("a time-domain plan searches float32 series only");
        return FDAS_E_INVAL;
    }
    auto mark = [&](int i) -> hipError_t { return timed ? hipEventRecord(p->tev[size_t(i)], st) : hipSuccess; };
    hipError_t e = mark(0);
    const float *x = static_cast<const float *>(in_dev);
    for (int32_t iz = 0; iz < p->nz && e == hipSuccess; ++iz) {
        const double alpha = row_value(p, iz);
        e = launch_td_resample(x, g.nsamp, alpha, ws.resampled, st);
        if (e == hipSuccess) e = launch_r2c_packed(ws.resampled, g.nsamp, ws.Z, ws.work, st);
        if (e == hipSuccess) e = launch_unpack_median(ws.Z, g.nsamp, ws.X, ws.med, p->W, st);
        if (e == hipSuccess)
            e = launch_td_power(ws.X, ws.med, p->W, g.nb, plane + int64_t(iz) * g.nb, ws.codes + int64_t(iz) * (g.nb / 2),
                                p->code_inv, st);
    }
    if (e != hipSuccess) return hip_fail(p, e, "time-domain spectra");
    for (int i = 1; i <= 4 && e == hipSuccess; ++i) e = mark(i);
    if (e == hipSuccess) e = launch_zero_u32(dcount, 6, st);
    if (e == hipSuccess)
        e = launch_harmsum(plane, ws.codes, p->nz, g.nb, 0, -1, p->opts.nharm_max, p->thr_f, p->code_thr, ws.hits,
                           p->hit_cap, p->group_cap, dcands, dcount, p->cand_cap, st);
    if (e == hipSuccess)
        e = launch_finish_candidates(dcands, dcount, p->cand_cap, ws.sort, p->nz, g.nb, 1, p->zmax, p->dz, ws.final, st);
    if (e == hipSuccess) e = launch_td_drift(dcount, p->cand_cap, p->zmax, p->nz, ws.final, st);
    for (int i = 5; i <= FDAS_NSTAGES && e == hipSuccess; ++i) e = mark(i);
    if (e != hipSuccess) return hip_fail(p, e, "time-domain harmonic sums");
    return FDAS_OK;
}

// Run the whole per-series path on `st`, writing the plane into `plane` and
// candidates into the plan's device buffers (count at *dcount).
double row_value(const fdas_plan_s *p, int32_t iz) {
    if (p->td && p->nz == 1) return 0.0;
    return -p->zmax + p->dz * double(iz);
}

fdas_status enqueue_search(fdas_plan_s *p, const Workspace &ws, const Geometry &g, int32_t in_kind,
                           const void *in_dev, float *plane, DevCand *dcands, uint32_t *dcount,
                           hipStream_t st, bool timed, const float2 **X_out, const double **med_out,
                           const DirectOut *direct) {
    if (X_out) *X_out = nullptr;
    if (med_out) *med_out = nullptr;
    if (p->td) return enqueue_td_search(p, ws, g, in_kind, in_dev, plane, dcands, dcount, st, timed);
    hipError_t e;
    const float2 *X = nullptr;
    const double *med = nullptr;
    // event i is recorded before stage i (and event FDAS_NSTAGES after the last)
    auto mark = [&](int i) -> hipError_t { return timed ? hipEventRecord(p->tev[size_t(i)], st) : hipSuccess; };
    if ((e = mark(0)) != hipSuccess) return hip_fail(p, e, "timing event");
    if (in_kind == FDAS_IN_SERIES_F32) {
        e = launch_r2c_packed(static_cast<const float *>(in_dev), g.nsamp, ws.Z, ws.work, st);
        if (e != hipSuccess) return hip_fail(p, e, "real-input DFT");
        if ((e = mark(1)) != hipSuccess) return hip_fail(p, e, "timing event");
        e = launch_unpack_median(ws.Z, g.nsamp, ws.X, ws.med, p->W, st);
        if (e != hipSuccess) return hip_fail(p, e, "unpack/median");
        X = ws.X;
        med = ws.med;
    } else if (in_kind == FDAS_IN_SPECTRUM_C64) {
        if ((e = mark(1)) != hipSuccess) return hip_fail(p, e, "timing event");
        X = static_cast<const float2 *>(in_dev);
        e = launch_median(X, g.nb, ws.med, p->W, st);
        if (e != hipSuccess) return hip_fail(p, e, "median");
        med = ws.med;
    } else {
        if ((e = mark(1)) != hipSuccess) return hip_fail(p, e, "timing event");
        X = static_cast<const float2 *>(in_dev);
    }
    if ((e = mark(2)) != hipSuccess) return hip_fail(p, e, "timing event");
    if (p->corr == FDAS_CORR_FFT_F32) {
        e = launch_segfft(X, med, p->W, g.nb, p->log2s, p->h, g.nseg, ws.seg, st);
        if (e != hipSuccess) return hip_fail(p, e, "segment DFT");
        if ((e = mark(3)) != hipSuccess) return hip_fail(p, e, "timing event");
        e = launch_correlate(ws.seg, p->d_bank, p->d_bank_half, p->nz, p->tpb, g.nb, p->log2s, p->h, g.nseg, plane,
                             ws.codes,
                             p->code_inv, st);
        if (e != hipSuccess) return hip_fail(p, e, "correlate");
    } else {
        const bool bf16 = p->corr == FDAS_CORR_GEMM_BF16;
        e = launch_lowp_spectrum(X, med, p->W, g.nb, bf16, ws.xl, st);
        if (e != hipSuccess) return hip_fail(p, e, "16-bit spectrum");
        if ((e = mark(3)) != hipSuccess) return hip_fail(p, e, "timing event");
        e = launch_corr_gemm(ws.xl, g.nb, p->h, p->d_gemm, p->nz, bf16, p->num_cu, plane, ws.codes, p->code_inv, st);
        if (e != hipSuccess) return hip_fail(p, e, "matrix correlate");
    }
    if ((e = mark(4)) != hipSuccess) return hip_fail(p, e, "timing event");
    e = launch_zero_u32(dcount, 6, st);
    if (e != hipSuccess) return hip_fail(p, e, "zero counter");
    e = launch_harmsum(plane, ws.codes, p->nz, g.ncol, p->opts.interbin ? g.nb : 0, p->izc, p->opts.nharm_max, p->thr_f, p->code_thr, ws.hits,
                       p->hit_cap, p->group_cap, dcands, dcount, p->cand_cap, st);
    if (e != hipSuccess) return hip_fail(p, e, "harmonic sum");
    if (direct && (p->td || p->opts.refine_levels > 0)) {
        set_error("records written to the host directly need a plan without refinement");
        return FDAS_E_INVAL;
    }
    e = direct ? launch_finish_candidates(dcands, dcount, p->cand_cap, ws.sort, p->nz, g.ncol, cols_per_bin(p), p->zmax,
                                          p->dz, direct->out, st, direct->cap, direct->count)
               : launch_finish_candidates(dcands, dcount, p->cand_cap, ws.sort, p->nz, g.ncol, cols_per_bin(p), p->zmax,
                                          p->dz, ws.final, st);
    if (e != hipSuccess) return hip_fail(p, e, "candidate sort");
    if ((e = mark(5)) != hipSuccess) return hip_fail(p, e, "timing event");
    if (p->opts.refine_levels > 0) {
        // four workgroups per compute unit, looping over the records
        e = launch_refine(X, med, p->W, g.nb, p->h, p->izc, p->dz, p->zmax, cols_per_bin(p), p->opts.refine_levels,
                          dcount, p->cand_cap, ws.final, 4 * p->num_cu, st);
        if (e != hipSuccess) return hip_fail(p, e, "candidate refinement");
    }
    if ((e = mark(6)) != hipSuccess) return hip_fail(p, e, "timing event");
    if (X_out) *X_out = X;
    if (med_out) *med_out = med;
    return FDAS_OK;
}

// Add the stage times of the last timed search (its events have completed).
fdas_status accumulate_timing(fdas_plan_s *p) {
    for (int i = 0; i < FDAS_NSTAGES; ++i) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, p->tev[size_t(i)], p->tev[size_t(i) + 1]);
        if (e != hipSuccess) return hip_fail(p, e, "stage timing");
        p->stage_ms[size_t(i)] += ms;
    }
    ++p->timed;
    return FDAS_OK;
}

// The status of a finished search from its counters in *ws.h_count (the
// records already copied).
static fdas_status count_status(const fdas_plan_s *p, const Workspace &ws, int64_t cap, int64_t *ncands) {
    const uint32_t found = ws.h_count[0];
    const bool hits_lost = ws.h_count[2] != 0;
    if (ncands) *ncands = found;
    if (hits_lost) {
        set_error("harmonic-sum cell list capacity exceeded: candidates incomplete (raise cand_capacity)");
        return FDAS_E_OVERFLOW;
    }
    if (int64_t(found) > cap || found > p->cand_cap) {
        set_error("candidate capacity exceeded");
        return FDAS_E_OVERFLOW;
    }
    return FDAS_OK;
}

fdas_status copy_candidates(const fdas_plan_s *p, const Workspace &ws, fdas_cand *out, int64_t cap,
                            int64_t *ncands, hipStream_t st) {
    const uint32_t found = ws.h_count[0];
    const bool hits_lost = ws.h_count[2] != 0;
    const int64_t n = std::min<int64_t>(std::min<int64_t>(found, p->cand_cap), cap);
    if (n > 0) {
        hipError_t e = hipMemcpyAsync(out, ws.final, size_t(n) * sizeof(fdas_cand), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(const_cast<fdas_plan_s *>(p), e, "copy candidates");
    }
    if (ncands) *ncands = found;
    if (hits_lost) {
        set_error("harmonic-sum cell list capacity exceeded: candidates incomplete (raise cand_capacity)");
        return FDAS_E_OVERFLOW;
    }
    if (int64_t(found) > cap || found > p->cand_cap) {
        set_error("candidate capacity exceeded");
        return FDAS_E_OVERFLOW;
    }
    return FDAS_OK;
}

static void free_workspace(Workspace &ws) {
    if (ws.Z) (void)hipFree(ws.Z);
    if (ws.resampled) (void)hipFree(ws.resampled);
    if (ws.work) (void)hipFree(ws.work);
    if (ws.X) (void)hipFree(ws.X);
    if (ws.med) (void)hipFree(ws.med);
    if (ws.seg) (void)hipFree(ws.seg);
    if (ws.plane) (void)hipFree(ws.plane);
    if (ws.codes) (void)hipFree(ws.codes);
    if (ws.xl) (void)hipFree(ws.xl);
    if (ws.cands) (void)hipFree(ws.cands);
    if (ws.count) (void)hipFree(ws.count);
    if (ws.sort) (void)hipFree(ws.sort);
    if (ws.hits) (void)hipFree(ws.hits);
    if (ws.final) (void)hipFree(ws.final);
    if (ws.h_count) (void)hipHostFree(ws.h_count);
    if (ws.series) (void)hipFree(ws.series);
    ws = Workspace{};
}

fdas_status alloc_workspace(fdas_plan_s *p, Workspace &ws, int64_t nsamp) {
    const Geometry g = make_geometry(nsamp, p->S, p->h, p->W, cols_per_bin(p));
    const int64_t M = g.nb;
    hipError_t e;
#define FDAS_ALLOC(ptr, bytes)                                                      \
    do {                                                                            \
        e = hipMalloc(reinterpret_cast<void **>(&(ptr)), size_t(bytes));            \
        if (e != hipSuccess) {                                                      \
            (void)hipGetLastError(); /* a failed allocation must not fail later launches */ \
            free_workspace(ws);                                                     \
            set_error(std::string("hipMalloc ") + #ptr + ": " + hipGetErrorString(e)); \
            return FDAS_E_NOMEM;                                                    \
        }                                                                           \
    } while (0)
    FDAS_ALLOC(ws.Z, M * 8);
    FDAS_ALLOC(ws.work, M * 8);
    FDAS_ALLOC(ws.X, M * 8);
    FDAS_ALLOC(ws.med, g.nblk * 8);
    if (p->td) FDAS_ALLOC(ws.resampled, nsamp * 4);
    else FDAS_ALLOC(ws.seg, g.nseg * int64_t(p->S) * 8);
    FDAS_ALLOC(ws.plane, int64_t(p->nz) * g.ncol * 4);
    FDAS_ALLOC(ws.codes, int64_t(p->nz) * (g.ncol / 2));
    if (p->corr != FDAS_CORR_FFT_F32) FDAS_ALLOC(ws.xl, g.nb * 4);
    FDAS_ALLOC(ws.cands, int64_t(p->cand_cap) * int64_t(sizeof(DevCand)));
    FDAS_ALLOC(ws.count, 64);
    FDAS_ALLOC(ws.sort, cand_sort_scratch_bytes(p->cand_cap));
    FDAS_ALLOC(ws.hits, harmsum_scratch_bytes(p->nz, g.ncol, p->hit_cap, p->group_cap));
    FDAS_ALLOC(ws.final, int64_t(p->cand_cap) * int64_t(sizeof(fdas_cand)));
#undef FDAS_ALLOC
    e = hipHostMalloc(reinterpret_cast<void **>(&ws.h_count), 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_workspace(ws);
        set_error("hipHostMalloc counter");
        return FDAS_E_NOMEM;
    }
    ws.nsamp = nsamp;
    return FDAS_OK;
}

void destroy_workspace(Workspace &ws) { free_workspace(ws); }

// Candidates of a search enqueued on st: counter, then records, to the host.
fdas_status collect(fdas_plan_s *p, Workspace &ws, fdas_cand *out, int64_t cap, int64_t *ncands,
                    hipStream_t st) {
    // Page-locked destination: one kernel writes the records and the counters
    // straight into host memory, with no round trip for the count in between.
    void *dev_out = nullptr, *dev_cnt = nullptr;
    if (cap > 0 && out && hipHostGetDevicePointer(&dev_out, out, 0) == hipSuccess && dev_out &&
        hipHostGetDevicePointer(&dev_cnt, ws.h_count, 0) == hipSuccess && dev_cnt) {
        const uint32_t c = uint32_t(std::min<int64_t>(cap, int64_t(p->cand_cap)));
        hipError_t e = launch_copy_records(ws.final, ws.count, c, static_cast<fdas_cand *>(dev_out),
                                           static_cast<uint32_t *>(dev_cnt), st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(p, e, "copy candidates");
        return count_status(p, ws, cap, ncands);
    }
    (void)hipGetLastError();  // a pageable destination is not an error
    hipError_t e = hipMemcpyAsync(ws.h_count, ws.count, 24, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(p, e, "copy candidate count");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(p, e, "search");
    return copy_candidates(p, ws, out, cap, ncands, st);
}

// Candidate capacities, thresholds and screening codes of a plan whose plane
// has cells_plane cells.
void init_detection(fdas_plan_s *p, int64_t cells_plane) {
    const fdas_opts &o = p->opts;
    p->cand_cap = uint32_t(o.cand_capacity > 0
                               ? o.cand_capacity
                               : std::min<int64_t>(int64_t(1) << 22, std::max<int64_t>(int64_t(1) << 16, cells_plane / 256)));
    // Bins the harmonic-sum screen may pass on: 4 x the candidate capacity,
    // and with the automatic capacity at least every bin of planes up to 2^24
    // bins (dense low-threshold searches flag most blocks).
    int64_t cells = int64_t(p->cand_cap) * 4;
    if (o.cand_capacity <= 0) cells = std::max<int64_t>(cells, std::min<int64_t>(cells_plane, int64_t(1) << 24));
    p->hit_cap = uint32_t(std::min<int64_t>(cells, int64_t(1) << 30));
    p->group_cap = std::max<uint32_t>(p->hit_cap / 2, 1u);
    int levels = 0;
    while ((1 << levels) < o.nharm_max) ++levels;
    for (int l = 0; l < 5; ++l) {
        p->thr_d[l] = l <= levels ? threshold(o.sigma, 1 << l) : INFINITY;
        p->thr_f[l] = float(p->thr_d[l]);
    }
    // Screening codes: delta = thr_max / 250, so a saturated code (255) clears
    // every level.  An exact FP32 sum S >= thr_f has code sum >= S / delta up to
    // a few roundings (< 2e-6 relative), hence >= floor(thr_f / delta (1 - 1e-5)).
    // Thresholds near zero (very low sigma) make every cell pass the screen.
    const double inv = 250.0 / double(p->thr_f[levels]);
    const bool screen = inv > 0.0 && inv < 1e30;
    p->code_inv = screen ? float(inv) : 1.f;
    for (int l = 0; l < 5; ++l) {
        const double t = double(p->thr_f[l]) * double(p->code_inv) * (1.0 - 1e-5);
        p->code_thr[l] = l > levels ? 0x8000u : screen && t > 0.0 ? uint32_t(std::floor(t)) : 0u;
    }
}

fdas_status make_plan_core(const fdas_bank_s *bank, int64_t nsamp, int32_t seg, const fdas_opts *opts,
                           fdas_plan_s **out) {
    *out = nullptr;
    if (!bank) {
        set_error("bank is NULL");
        return FDAS_E_INVAL;
    }
    fdas_opts o;
    if (opts) o = *opts; else fdas_default_opts(&o);
    fdas_status st = validate_opts(o);
    if (st != FDAS_OK) return st;
    st = check_nsamp(nsamp, seg, bank->h);
    if (st != FDAS_OK) return st;
    if (!is_pow2(seg) || seg < 256 || seg > 8192 || seg < 4 * bank->h) {
        set_error("seg must be a power of two in [256, 8192] and >= 4h");
        return FDAS_E_INVAL;
    }
    if (nsamp / 2 < int64_t(o.median_window)) {
        set_error("nsamp / 2 must be at least the median window");
        return FDAS_E_INVAL;
    }
    auto *p = new (std::nothrow) fdas_plan_s;
    if (!p) {
        set_error("out of host memory");
        return FDAS_E_NOMEM;
    }
    p->opts = o;
    p->zmax = bank->zmax;
    p->dz = bank->dz;
    p->nz = bank->nz;
    p->h = bank->h;
    p->izc = (bank->nz - 1) / 2;
    p->S = seg;
    p->log2s = ilog2(seg);
    p->W = o.median_window;
    p->nsamp = nsamp;
    p->tpb = o.templates_per_block > 0 ? o.templates_per_block : default_tpb(bank->nz);
    p->corr = o.correlator;
    if (p->corr != FDAS_CORR_FFT_F32 && gemm_ksteps(bank->h) > GM_MAX_KSTEPS) {
        delete p;
        set_error("the matrix correlators need h <= 271 (zmax <= 510)");
        return FDAS_E_INVAL;
    }
    init_detection(p, int64_t(bank->nz) * (nsamp / 2) * cols_per_bin(p));
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        set_error(std::string("no HIP device: ") + hipGetErrorString(e));
        return FDAS_E_DEVICE;
    }
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && ncu > 0)
            p->num_cu = ncu;
    }
    if (p->corr != FDAS_CORR_FFT_F32) {
        // Template matrix of the matrix correlator (16-bit, fragment order).
        std::vector<uint8_t> gm(gemm_bank_bytes(p->nz, p->h));
        build_gemm_bank(reinterpret_cast<const double *>(bank->taps.data()), p->nz, p->h,
                        p->corr == FDAS_CORR_GEMM_BF16, gm.data());
        e = hipMalloc(&p->d_gemm, gm.size());
        if (e == hipSuccess) e = hipMemcpy(p->d_gemm, gm.data(), gm.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (p->d_gemm) (void)hipFree(p->d_gemm);
            delete p;
            set_error(std::string("template matrix: ") + hipGetErrorString(e));
            return FDAS_E_NOMEM;
        }
        *out = p;
        return FDAS_OK;
    }
    // Template bank in the segment domain: taps wrapped circularly (q >= 0 at
    // n = q, q < 0 at n = S + q), FP64 DFT, times 1/S, rounded to float32.
    // With interbin a second bank holds the taps of the half-bin offsets.
    const int32_t S = seg, ntap = 2 * p->h + 1;
    std::vector<float2> host(size_t(p->nz) * S);
    std::vector<cd> t(S), htaps(static_cast<size_t>(ntap));
    auto to_segment_domain = [&](const cd *taps, int32_t iz) {
        std::fill(t.begin(), t.end(), cd(0.0, 0.0));
        for (int32_t q = -p->h; q <= p->h; ++q) t[size_t((q + S) % S)] = taps[q + p->h];
        fft_inplace(t, -1);
        for (int32_t f = 0; f < S; ++f) {
            const cd v = t[size_t(f)] / double(S);
            host[size_t(iz) * S + f] = make_float2(float(v.real()), float(v.imag()));
        }
    };
    auto upload = [&](float2 **dst, const char *what) -> fdas_status {
        hipError_t er = hipMalloc(reinterpret_cast<void **>(dst), host.size() * sizeof(float2));
        if (er != hipSuccess) {
            (void)hipGetLastError();
            *dst = nullptr;
            set_error(std::string("hipMalloc ") + what + ": " + hipGetErrorString(er));
            return FDAS_E_NOMEM;
        }
        er = hipMemcpy(*dst, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice);
        if (er != hipSuccess) {
            set_error(std::string("upload ") + what + ": " + hipGetErrorString(er));
            return FDAS_E_DEVICE;
        }
        return FDAS_OK;
    };
    auto fail = [&](fdas_status st) {
        if (p->d_bank) (void)hipFree(p->d_bank);
        if (p->d_bank_half) (void)hipFree(p->d_bank_half);
        delete p;
        return st;
    };
    for (int32_t iz = 0; iz < p->nz; ++iz) to_segment_domain(&bank->taps[size_t(iz) * ntap], iz);
    fdas_status ust = upload(&p->d_bank, "bank");
    if (ust != FDAS_OK) return fail(ust);
    if (o.interbin) {
        for (int32_t iz = 0; iz < p->nz; ++iz) {
            template_taps_half(fdas_bank_z(bank, iz), p->h, htaps.data());
            to_segment_domain(htaps.data(), iz);
        }
        ust = upload(&p->d_bank_half, "half-bin bank");
        if (ust != FDAS_OK) return fail(ust);
    }
    *out = p;
    return FDAS_OK;
}
}  // namespace fdas

using namespace fdas;

extern "C" {

void fdas_default_opts(fdas_opts *opts) {
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->sigma = 6.0;
    opts->nharm_max = 16;
    opts->median_window = 1024;
    opts->cand_capacity = 0;
    opts->templates_per_block = 0;
}

fdas_status fdas_make_templates(double zmax, double dz, fdas_bank **out) {
    if (!out) {
        set_error("out is NULL");
        return FDAS_E_INVAL;
    }
    *out = nullptr;
    if (!(zmax >= 0.0 && zmax <= 1200.0) || !(dz > 0.0)) {
        set_error("need 0 <= zmax <= 1200 and dz > 0");
        return FDAS_E_INVAL;
    }
    const double ratio = 2.0 * zmax / dz;
    const double rr = std::nearbyint(ratio);
    if (std::fabs(ratio - rr) > 1e-9 * std::max(1.0, ratio) || rr > 4800.0) {
        set_error("2 zmax / dz must be an integer <= 4800");
        return FDAS_E_INVAL;
    }
    auto *b = new (std::nothrow) fdas_bank_s;
    if (!b) {
        set_error("out of host memory");
        return FDAS_E_NOMEM;
    }
    b->zmax = zmax;
    b->dz = dz;
    b->nz = int32_t(rr) + 1;
    b->h = template_halfwidth(zmax);
    const int32_t ntap = 2 * b->h + 1;
    b->taps.resize(size_t(b->nz) * ntap);
    for (int32_t iz = 0; iz < b->nz; ++iz) template_taps(-zmax + double(iz) * dz, b->h, &b->taps[size_t(iz) * ntap]);
    *out = b;
    return FDAS_OK;
}

int32_t fdas_bank_nz(const fdas_bank *bank) { return bank ? bank->nz : 0; }
int32_t fdas_bank_halfwidth(const fdas_bank *bank) { return bank ? bank->h : 0; }
double fdas_bank_z(const fdas_bank *bank, int32_t iz) {
    return bank ? -bank->zmax + double(iz) * bank->dz : 0.0;
}

fdas_status fdas_bank_taps(const fdas_bank *bank, int32_t iz, double *re_im_out) {
    if (!bank || !re_im_out || iz < 0 || iz >= bank->nz) {
        set_error("bad bank, output or template index");
        return FDAS_E_INVAL;
    }
    const int32_t ntap = 2 * bank->h + 1;
    for (int32_t i = 0; i < ntap; ++i) {
        const cd v = bank->taps[size_t(iz) * ntap + i];
        re_im_out[2 * i] = v.real();
        re_im_out[2 * i + 1] = v.imag();
    }
    return FDAS_OK;
}

void fdas_bank_destroy(fdas_bank *bank) { delete bank; }

fdas_status fdas_threshold(double sigma, int32_t nharm, double *thr) {
    if (!thr || nharm < 1 || nharm > 64 || !(sigma > -30.0 && sigma < 1000.0)) {
        set_error("bad threshold arguments");
        return FDAS_E_INVAL;
    }
    *thr = threshold(sigma, nharm);
    return FDAS_OK;
}

fdas_status fdas_significance(double power, int32_t nharm, double *sigma) {
    if (!sigma || nharm < 1 || nharm > 64 || !(power >= 0.0) || !std::isfinite(power)) {
        set_error("bad significance arguments");
        return FDAS_E_INVAL;
    }
    *sigma = significance(power, nharm);
    return FDAS_OK;
}

fdas_status fdas_plan(const fdas_bank *bank, int64_t nsamp, int32_t seg, const fdas_opts *opts,
                      fdas_plan_t **out) {
    if (!out) {
        set_error("out is NULL");
        return FDAS_E_INVAL;
    }
    *out = nullptr;
    fdas_plan_s *p = nullptr;
    fdas_status st = make_plan_core(bank, nsamp, seg, opts, &p);
    if (st != FDAS_OK) return st;
    st = alloc_workspace(p, p->ws[0], nsamp);
    if (st != FDAS_OK) {
        fdas_plan_destroy(p);
        return st;
    }
    *out = p;
    return FDAS_OK;
}

fdas_status fdas_td_plan(int64_t nsamp, double alpha_max, int32_t nalpha, const fdas_opts *opts,
                         fdas_plan_t **out) {
    if (!out) {
        set_error("out is NULL");
        return FDAS_E_INVAL;
    }
    *out = nullptr;
    fdas_opts o;
    if (opts) o = *opts; else fdas_default_opts(&o);
    fdas_status st = validate_opts(o);
    if (st != FDAS_OK) return st;
    if (o.correlator != FDAS_CORR_FFT_F32 || o.interbin || o.refine_levels) {
        set_error("a time-domain plan takes no correlator, half-bin plane or refinement options");
        return FDAS_E_INVAL;
    }
    st = check_nsamp(nsamp, 0, 0);
    if (st != FDAS_OK) return st;
    if (nsamp / 2 < int64_t(o.median_window)) {
        set_error("nsamp / 2 must be at least the median window");
        return FDAS_E_INVAL;
    }
    if (nalpha < 1 || nalpha > 4801 || !(alpha_max >= 0.0 && alpha_max <= 0.5)) {
        set_error("nalpha must be in [1, 4801] and alpha_max in [0, 0.5]");
        return FDAS_E_INVAL;
    }
    auto *p = new (std::nothrow) fdas_plan_s;
    if (!p) {
        set_error("out of host memory");
        return FDAS_E_NOMEM;
    }
    p->opts = o;
    p->td = true;
    p->zmax = alpha_max;
    p->dz = nalpha > 1 ? 2.0 * alpha_max / double(nalpha - 1) : 0.0;
    p->nz = nalpha;
    p->h = 0;
    p->izc = -1;
    p->S = 0;
    p->log2s = 0;
    p->W = o.median_window;
    p->nsamp = nsamp;
    p->tpb = 1;
    p->corr = FDAS_CORR_FFT_F32;
    init_detection(p, int64_t(nalpha) * (nsamp / 2));
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        set_error(std::string("no HIP device: ") + hipGetErrorString(e));
        return FDAS_E_DEVICE;
    }
    st = alloc_workspace(p, p->ws[0], nsamp);
    if (st != FDAS_OK) {
        fdas_plan_destroy(p);
        return st;
    }
    *out = p;
    return FDAS_OK;
}

int64_t fdas_plan_nbins(const fdas_plan_t *plan) { return plan ? plan->nsamp / 2 : 0; }

int32_t fdas_plan_rows(const fdas_plan_t *plan) { return plan ? plan->nz : 0; }

double fdas_plan_row_value(const fdas_plan_t *plan, int32_t iz) {
    if (!plan || iz < 0 || iz >= plan->nz) return NAN;
    return row_value(plan, iz);
}

int64_t fdas_plan_device_bytes(const fdas_plan_t *plan) {
    if (!plan) return 0;
    int64_t b = plan->td ? 0
                : plan->corr == FDAS_CORR_FFT_F32 ? int64_t(plan->nz) * plan->S * 8 * cols_per_bin(plan)
                                                  : int64_t(gemm_bank_bytes(plan->nz, plan->h));
    for (const Workspace &ws : plan->ws) {
        if (ws.nsamp) {
            const Geometry g = make_geometry(ws.nsamp, plan->S, plan->h, plan->W, cols_per_bin(plan));
            b += series_bytes(g, plan->S, plan->nz) + candidate_bytes(plan, g);
            if (plan->td) b += ws.nsamp * 4;  // the resampled series
        }
    }
    return b;
}

void fdas_plan_destroy(fdas_plan_t *plan) {
    if (!plan) return;
    if (plan->copy_stream) {
        (void)hipStreamSynchronize(plan->copy_stream);  // a prefetch may still write in_dev
        (void)hipStreamDestroy(plan->copy_stream);
    }
    for (float *&b : plan->in_dev) {
        if (b) (void)hipFree(b);
        b = nullptr;
    }
    for (hipEvent_t &ev : plan->in_ready) {
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
    }
    for (Workspace &ws : plan->ws) destroy_workspace(ws);
    for (hipStream_t &s : plan->aux) {
        if (s) (void)hipStreamDestroy(s);
        s = nullptr;
    }
    for (hipEvent_t &ev : plan->events) {
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
    }
    for (hipEvent_t &ev : plan->tev) {
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
    }
    for (auto &m : plan->graphs)
        for (auto &kv : m) (void)hipGraphExecDestroy(kv.second);
    destroy_pbatch(plan->pbatch);
    plan->pbatch = nullptr;
    if (plan->d_bank) (void)hipFree(plan->d_bank);
    if (plan->d_bank_half) (void)hipFree(plan->d_bank_half);
    if (plan->d_gemm) (void)hipFree(plan->d_gemm);
    delete plan;
}

fdas_status fdas_search(fdas_plan_t *plan, int32_t in_kind, const void *in_dev, float *plane_dev,
                        fdas_cand *cands_host, int64_t cap, int64_t *ncands, void *hip_stream) {
    if (!plan || !in_dev || cap < 0 || (cap > 0 && !cands_host)) {
        set_error("bad plan, input or candidate buffer");
        return FDAS_E_INVAL;
    }
    if (in_kind < FDAS_IN_SERIES_F32 || in_kind > FDAS_IN_SPECTRUM_C64_NORMALISED) {
        set_error("bad input kind");
        return FDAS_E_INVAL;
    }
    if (reinterpret_cast<uintptr_t>(plane_dev) % 16 != 0) {
        set_error("plane_dev must be 16-byte aligned");
        return FDAS_E_INVAL;
    }
    if (plan->broken) {
        set_error("plan is unusable after a device error");
        return FDAS_E_DEVICE;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Workspace &ws = plan->ws[0];
    const Geometry g = make_geometry(plan->nsamp, plan->S, plan->h, plan->W, cols_per_bin(plan));
    float *plane = plane_dev ? plane_dev : ws.plane;
    const bool timed = plan->timing;
    const float2 *X = nullptr;
    const double *med = nullptr;
    plan->searched = false;
    plan->last_X = nullptr;
    plan->last_med = nullptr;
    // Page-locked destination and nothing to post-process: the finishing
    // kernel writes the records and the counters straight into host memory.
    DirectOut direct{};
    bool use_direct = false;
    if (cap > 0 && !plan->td && plan->opts.refine_levels == 0) {
        void *dev_out = nullptr, *dev_cnt = nullptr;
        if (hipHostGetDevicePointer(&dev_out, cands_host, 0) == hipSuccess && dev_out &&
            hipHostGetDevicePointer(&dev_cnt, ws.h_count, 0) == hipSuccess && dev_cnt) {
            direct = DirectOut{static_cast<fdas_cand *>(dev_out), uint32_t(std::min<int64_t>(cap, plan->cand_cap)),
                               static_cast<uint32_t *>(dev_cnt)};
            use_direct = true;
        }
        (void)hipGetLastError();  // a pageable destination is not an error
    }
    fdas_status s = enqueue_search(plan, ws, g, in_kind, in_dev, plane, ws.cands, ws.count, st, timed, &X, &med,
                                   use_direct ? &direct : nullptr);
    if (s != FDAS_OK) return s;
    plan->last_X = X;
    plan->last_med = med;
    plan->last_nb = g.nb;
    plan->searched = true;
    if (use_direct) {
        const hipError_t e = hipStreamSynchronize(st);
        s = e != hipSuccess ? hip_fail(plan, e, "search") : count_status(plan, ws, cap, ncands);
    } else {
        s = collect(plan, ws, cands_host, cap, ncands, st);
    }
    if (timed && (s == FDAS_OK || s == FDAS_E_OVERFLOW)) {
        const fdas_status t = accumulate_timing(plan);
        if (t != FDAS_OK) return t;
    }
    return s;
}

fdas_status fdas_search_host(fdas_plan_t *plan, const float *series_host, const float *next_host,
                             float *plane_dev, fdas_cand *cands_host, int64_t cap, int64_t *ncands,
                             void *hip_stream) {
    if (!plan || !series_host || cap < 0 || (cap > 0 && !cands_host)) {
        set_error("bad plan, host series or candidate buffer");
        return FDAS_E_INVAL;
    }
    if (reinterpret_cast<uintptr_t>(plane_dev) % 16 != 0) {
        set_error("plane_dev must be 16-byte aligned");
        return FDAS_E_INVAL;
    }
    if (plan->broken) {
        set_error("plan is unusable after a device error");
        return FDAS_E_DEVICE;
    }
    const size_t bytes = size_t(plan->nsamp) * sizeof(float);
    hipError_t e = hipSuccess;
    if (!plan->copy_stream) {
        for (float *&b : plan->in_dev) {
            e = hipMalloc(reinterpret_cast<void **>(&b), bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                for (float *&x : plan->in_dev) {
                    if (x) (void)hipFree(x);
                    x = nullptr;
                }
                set_error("hipMalloc host-series input buffers");
                return FDAS_E_NOMEM;
            }
        }
        for (hipEvent_t &ev : plan->in_ready) {
            if (!ev && (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(plan, e, "event create");
        }
        if ((e = hipStreamCreateWithFlags(&plan->copy_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(plan, e, "copy stream create");
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int slot;
    if (plan->staged_slot >= 0 && plan->staged_host == series_host) {
        // the previous call started this copy on the copy stream
        slot = plan->staged_slot;
        if ((e = hipStreamWaitEvent(st, plan->in_ready[size_t(slot)], 0)) != hipSuccess)
            return hip_fail(plan, e, "wait for the staged series");
    } else {
        // a staged series that is not used is dropped once its copy is done
        slot = plan->staged_slot >= 0 ? plan->staged_slot : 0;
        if (plan->staged_slot >= 0 && (e = hipStreamWaitEvent(st, plan->in_ready[size_t(slot)], 0)) != hipSuccess)
            return hip_fail(plan, e, "wait for the staged series");
        if ((e = hipMemcpyAsync(plan->in_dev[size_t(slot)], series_host, bytes, hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return hip_fail(plan, e, "copy series to the device");
    }
    plan->staged_host = nullptr;
    plan->staged_slot = -1;
    if (next_host) {
        // every earlier search has returned (each call ends with a stream
        // synchronisation), so the other buffer is no longer read
        const int ns = 1 - slot;
        if ((e = hipMemcpyAsync(plan->in_dev[size_t(ns)], next_host, bytes, hipMemcpyHostToDevice,
                                plan->copy_stream)) != hipSuccess ||
            (e = hipEventRecord(plan->in_ready[size_t(ns)], plan->copy_stream)) != hipSuccess)
            return hip_fail(plan, e, "start the next series' copy");
        plan->staged_host = next_host;
        plan->staged_slot = ns;
    }
    return fdas_search(plan, FDAS_IN_SERIES_F32, plan->in_dev[size_t(slot)], plane_dev, cands_host, cap, ncands,
                       hip_stream);
}

fdas_status fdas_plan_enable_timing(fdas_plan_t *plan, int32_t enable) {
    if (!plan) {
        set_error("plan is NULL");
        return FDAS_E_INVAL;
    }
    for (hipEvent_t &ev : plan->tev) {
        if (!ev) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_fail(plan, e, "event create");
        }
    }
    plan->timing = enable != 0;
    plan->stage_ms.fill(0.0);
    plan->timed = 0;
    return FDAS_OK;
}

fdas_status fdas_plan_stage_times(const fdas_plan_t *plan, double *ms_out, int64_t *nsearch_out) {
    if (!plan || !ms_out) {
        set_error("plan or output is NULL");
        return FDAS_E_INVAL;
    }
    for (int i = 0; i < FDAS_NSTAGES; ++i) ms_out[i] = plan->stage_ms[size_t(i)];
    if (nsearch_out) *nsearch_out = plan->timed;
    return FDAS_OK;
}

fdas_status fdas_plan_search_counts(const fdas_plan_t *plan, int64_t *out3) {
    if (!plan || !out3) {
        set_error("plan or output is NULL");
        return FDAS_E_INVAL;
    }
    const uint32_t *c = plan->ws[0].h_count;
    if (!c || !plan->searched) {
        set_error("no search has run on this plan");
        return FDAS_E_INVAL;
    }
    out3[0] = c[0];
    out3[1] = c[4];
    out3[2] = c[5];
    return FDAS_OK;
}

fdas_status fdas_plan_fetch_spectrum(fdas_plan_t *plan, void *spectrum_dev, double *medians_dev, void *hip_stream) {
    if (!plan || !plan->last_X) {
        set_error("no search has run on this plan");
        return FDAS_E_INVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t nb = plan->last_nb;
    hipError_t e;
    if (spectrum_dev) {
        if (plan->last_med)
            e = launch_normalise(plan->last_X, plan->last_med, plan->W, nb, static_cast<float2 *>(spectrum_dev), st);
        else
            e = hipMemcpyAsync(spectrum_dev, plan->last_X, size_t(nb) * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(plan, e, "fetch spectrum");
    }
    if (medians_dev && plan->last_med) {
        e = hipMemcpyAsync(medians_dev, plan->last_med, size_t((nb + plan->W - 1) / plan->W) * 8,
                           hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(plan, e, "fetch medians");
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(plan, e, "fetch");
    return FDAS_OK;
}

fdas_status fdas_interp_power(fdas_plan_t *plan, int64_t n, const double *r, const double *z, const int32_t *nharm,
                              double *power_out, void *hip_stream) {
    if (plan && plan->td) {
        set_error("interpolation needs a template (FDAS) plan");
        return FDAS_E_INVAL;
    }
    if (!plan || !plan->last_X) {
        set_error("no search has run on this plan");
        return FDAS_E_INVAL;
    }
    if (n < 0 || n > (int64_t(1) << 31) || (n > 0 && (!r || !z || !nharm || !power_out))) {
        set_error("fdas_interp_power: n out of range or a NULL array");
        return FDAS_E_INVAL;
    }
    if (n == 0) return FDAS_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const size_t nd = size_t(n) * sizeof(double);
    char *buf = nullptr;
    hipError_t e = hipMalloc(&buf, 3 * nd + size_t(n) * sizeof(int32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("fdas_interp_power: device allocation failed");
        return FDAS_E_NOMEM;
    }
    double *dr = reinterpret_cast<double *>(buf);
    double *dzv = dr + n;
    double *dout = dzv + n;
    int32_t *dnh = reinterpret_cast<int32_t *>(dout + n);
    const int64_t nb = plan->last_nb;
    if ((e = hipMemcpyAsync(dr, r, nd, hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = hipMemcpyAsync(dzv, z, nd, hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = hipMemcpyAsync(dnh, nharm, size_t(n) * sizeof(int32_t), hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = launch_interp_points(plan->last_X, plan->last_med, plan->W, nb, plan->h, dr, dzv, dnh, n, dout, st)) ==
            hipSuccess &&
        (e = hipMemcpyAsync(power_out, dout, nd, hipMemcpyDeviceToHost, st)) == hipSuccess) {
        e = hipStreamSynchronize(st);
    }
    const hipError_t ef = hipFree(buf);
    if (e != hipSuccess) return hip_fail(plan, e, "interpolated power");
    if (ef != hipSuccess) return hip_fail(plan, ef, "free");
    return FDAS_OK;
}

// Argument checks shared by fdas_refine and fdas_refine_noalloc.
static fdas_status check_refine_args(const fdas_plan_t *plan, const fdas_cand *cands, int64_t n, int32_t levels) {
    if (plan && plan->td) {
        set_error("refinement needs a template (FDAS) plan");
        return FDAS_E_INVAL;
    }
    if (!plan || !plan->last_X) {
        set_error("no search has run on this plan");
        return FDAS_E_INVAL;
    }
    if (n < 0 || n > int64_t(UINT32_MAX) || (n > 0 && !cands) || levels < 1 || levels > 20) {
        set_error("fdas_refine: n out of range, NULL records or levels not in [1, 20]");
        return FDAS_E_INVAL;
    }
    for (int64_t i = 0; i < n; ++i) {
        const int32_t m = cands[i].nharm;
        if (m != 1 && m != 2 && m != 4 && m != 8 && m != 16) {
            set_error("fdas_refine: a record's nharm is not 1, 2, 4, 8 or 16");
            return FDAS_E_INVAL;
        }
    }
    return FDAS_OK;
}

// Records dc and count dn on the device (either buffer the caller provides):
// copy in, refine, copy back, wait.
static hipError_t refine_on_device(fdas_plan_t *plan, fdas_cand *cands, int64_t n, int32_t levels, fdas_cand *dc,
                                   uint32_t *dn, const uint32_t *nn_host, hipStream_t st) {
    const size_t bytes = size_t(n) * sizeof(fdas_cand);
    hipError_t e;
    if ((e = hipMemcpyAsync(dc, cands, bytes, hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = hipMemcpyAsync(dn, nn_host, sizeof(uint32_t), hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = launch_refine(plan->last_X, plan->last_med, plan->W, plan->last_nb, plan->h, plan->izc, plan->dz,
                           plan->zmax, cols_per_bin(plan), levels, dn, uint32_t(n), dc, 4 * plan->num_cu, st)) ==
            hipSuccess &&
        (e = hipMemcpyAsync(cands, dc, bytes, hipMemcpyDeviceToHost, st)) == hipSuccess) {
        e = hipStreamSynchronize(st);
    }
    return e;
}

fdas_status fdas_refine_noalloc(fdas_plan_t *plan, fdas_cand *cands, int64_t n, int32_t levels, void *hip_stream) {
    fdas_status s = check_refine_args(plan, cands, n, levels);
    if (s != FDAS_OK) return s;
    if (n > FDAS_REFINE_NOALLOC_MAX) {
        set_error("fdas_refine_noalloc: more than FDAS_REFINE_NOALLOC_MAX (16384) records; use fdas_refine");
        return FDAS_E_INVAL;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "fdas_refine_noalloc: current device");
    if (dev != plan->device) {
        set_error("fdas_refine_noalloc: the current device is not the plan's");
        return FDAS_E_INVAL;
    }
    if (n == 0) return FDAS_OK;
    void *scr = nullptr;
    size_t scr_bytes = 0;
    e = refine_noalloc_scratch(&scr, &scr_bytes);
    if (e != hipSuccess) return hip_fail(plan, e, "fdas_refine_noalloc: scratch address");
    fdas_cand *dc = static_cast<fdas_cand *>(scr);
    uint32_t *dn = reinterpret_cast<uint32_t *>(static_cast<char *>(scr) + size_t(FDAS_REFINE_NOALLOC_MAX) *
                                                                              sizeof(fdas_cand));
    if (size_t(FDAS_REFINE_NOALLOC_MAX) * sizeof(fdas_cand) + sizeof(uint32_t) > scr_bytes) {
        set_error("fdas_refine_noalloc: scratch array too small");
        return FDAS_E_DEVICE;
    }
    const uint32_t nn = uint32_t(n);
    e = refine_on_device(plan, cands, n, levels, dc, dn, &nn, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(plan, e, "refine");
    return FDAS_OK;
}

fdas_status fdas_refine(fdas_plan_t *plan, fdas_cand *cands, int64_t n, int32_t levels, void *hip_stream) {
    fdas_status s = check_refine_args(plan, cands, n, levels);
    if (s != FDAS_OK) return s;
    if (n == 0) return FDAS_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const size_t bytes = size_t(n) * sizeof(fdas_cand);
    char *buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes + sizeof(uint32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("fdas_refine: device allocation failed");
        return FDAS_E_NOMEM;
    }
    fdas_cand *dc = reinterpret_cast<fdas_cand *>(buf);
    uint32_t *dn = reinterpret_cast<uint32_t *>(buf + bytes);
    const uint32_t nn = uint32_t(n);
    e = refine_on_device(plan, cands, n, levels, dc, dn, &nn, st);
    const hipError_t ef = hipFree(buf);
    if (e != hipSuccess) return hip_fail(plan, e, "refine");
    if (ef != hipSuccess) return hip_fail(plan, ef, "free");
    return FDAS_OK;
}

fdas_status fdas_dedisperse(const uint8_t *fil_dev, int32_t nchan, int64_t nsamp, double f_top, double foff,
                            double tsamp, const double *dms, int32_t ndm, int64_t nout, float *out_dev,
                            void *hip_stream) {
    if (!fil_dev || !out_dev || !dms || (reinterpret_cast<uintptr_t>(fil_dev) & 3u) != 0 || nchan < 1 ||
        nchan > 65536 || ndm < 1 || ndm > 65536 || nsamp < 1 ||
        nout < 1 || !(tsamp > 0.0) || !(foff >= 0.0) || !(f_top - foff * double(nchan - 1) > 0.0) ||
        !std::isfinite(f_top)) {
        set_error("fdas_dedisperse: bad filterbank, frequency, sampling or DM arguments");
        return FDAS_E_INVAL;
    }
    // delays d[i][c] = floor(KDM DM_i (f_c^-2 - f_top^-2) / tsamp + 1/2), FP64
    constexpr double kKdm = 4.148808e3;  // s MHz^2 pc^-1 cm^3
    std::vector<int32_t> d(size_t(ndm) * size_t(nchan));
    int64_t dmax = 0;
    for (int32_t i = 0; i < ndm; ++i) {
        if (!(dms[i] >= 0.0) || !std::isfinite(dms[i])) {
            set_error("fdas_dedisperse: DMs must be finite and >= 0");
            return FDAS_E_INVAL;
        }
        for (int32_t c = 0; c < nchan; ++c) {
            const double f = f_top - foff * double(c);
            const double raw = kKdm * dms[i] * (1.0 / (f * f) - 1.0 / (f_top * f_top)) / tsamp;
            const double v = std::floor(raw + 0.5);
            if (!(v < double(nsamp)) || v > 2147483647.0) {
                set_error("fdas_dedisperse: a delay exceeds the filterbank (or 2^31 samples)");
                return FDAS_E_INVAL;
            }
            d[size_t(i) * nchan + c] = int32_t(v);
            dmax = std::max<int64_t>(dmax, int64_t(v));
        }
    }
    if (nout > nsamp - dmax) {
        set_error("fdas_dedisperse: nout exceeds nsamp minus the largest delay");
        return FDAS_E_INVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int32_t *dd = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&dd), d.size() * sizeof(int32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("fdas_dedisperse: device allocation failed");
        return FDAS_E_NOMEM;
    }
    if ((e = hipMemcpyAsync(dd, d.data(), d.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)) == hipSuccess &&
        (e = launch_dedisperse(fil_dev, nchan, nsamp, dd, ndm, nout, out_dev, st)) == hipSuccess)
        e = hipStreamSynchronize(st);
    const hipError_t ef = hipFree(dd);
    if (e != hipSuccess || ef != hipSuccess) {
        set_error(std::string("fdas_dedisperse: ") + hipGetErrorString(e != hipSuccess ? e : ef));
        return FDAS_E_DEVICE;
    }
    return FDAS_OK;
}

fdas_status fdas_dft_c64(int32_t log2n, int32_t inverse, int64_t batch, const void *in_dev, void *out_dev,
                         void *hip_stream) {
    if (log2n < 6 || log2n > 13 || batch < 0 || batch > 0x7fffffff || (batch > 0 && (!in_dev || !out_dev))) {
        set_error("bad DFT arguments");
        return FDAS_E_INVAL;
    }
    hipError_t e = launch_dft(log2n, inverse ? +1 : -1, batch, static_cast<const float2 *>(in_dev),
                              static_cast<float2 *>(out_dev), static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(nullptr, e, "dft");
    return FDAS_OK;
}

const char *fdas_strerror(fdas_status status) {
    switch (status) {
        case FDAS_OK: return "ok";
        case FDAS_E_INVAL: return "invalid argument";
        case FDAS_E_NOMEM: return "out of memory";
        case FDAS_E_DEVICE: return "device error";
        case FDAS_E_OVERFLOW: return "candidate capacity exceeded";
        case FDAS_E_BUSY: return "queue full";
        case FDAS_E_TIMEOUT: return "timed out";
    }
    return "unknown status";
}

const char *fdas_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
