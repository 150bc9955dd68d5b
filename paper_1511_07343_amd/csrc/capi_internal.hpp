// Internal state behind the C ABI: bank, plan, work buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/fdas.h"
#include "host_math.hpp"
#include "kernels.hpp"

struct fdas_bank_s {
    double zmax = 0.0, dz = 1.0;
    int32_t nz = 0, h = 0;
    std::vector<fdas::cd> taps;  // nz x (2h+1), tap q at column q + h
};

namespace fdas {

// Per-length geometry.
struct Geometry {
    int64_t nsamp = 0, nb = 0, L = 0, nseg = 0, nblk = 0;
    int64_t ncol = 0;  // plane columns: nb, or 2 nb for a half-bin plane
};

// Device buffers for one series in flight (sized for `nsamp`).
struct Workspace {
    int64_t nsamp = 0;
    float2 *Z = nullptr;     // complex DFT of the packed series, M = nsamp/2
    float2 *work = nullptr;  // four-step scratch, M
    float2 *X = nullptr;     // real-input spectrum, nb bins
    double *med = nullptr;   // block medians of |X|^2
    float2 *seg = nullptr;   // segment spectra, nseg x S
    float *plane = nullptr;  // f-fdot plane, nz x nb
    uint8_t *codes = nullptr;  // screening codes of the plane's 2-bin blocks, nz x nb/2
    uint32_t *xl = nullptr;    // 16-bit spectrum of the matrix correlator, nb words
    DevCand *cands = nullptr;     // unordered records from the harmonic-sum kernel
    uint32_t *count = nullptr;    // their count (may exceed the capacity)
    void *hits = nullptr;         // harmonic-sum screen lists, exact sums and group map
    void *sort = nullptr;         // radix-sort scratch
    fdas_cand *final = nullptr;   // sorted public records
    uint32_t *h_count = nullptr;  // pinned host copy of the count
    float *series = nullptr;      // graph input: the trial is copied here first (batched path)
    float *resampled = nullptr;   // time-domain search: the series resampled for one trial
};

}  // namespace fdas

namespace fdas {
struct PBatch;  // resources of the persistent batch launch (batch.cpp)
void destroy_pbatch(PBatch *pb);
}  // namespace fdas

struct fdas_plan_s {
    fdas_opts opts{};
    double zmax = 0.0, dz = 1.0;
    int32_t nz = 0, h = 0, izc = 0, S = 0, log2s = 0, W = 1024, tpb = 13;
    int64_t nsamp = 0;
    uint32_t cand_cap = 0;  // device candidate capacity (records)
    uint32_t hit_cap = 0;   // device capacity of the harmonic-sum screen's cell list
    uint32_t group_cap = 0; // ... and of its group list
    int device = 0;
    double thr_d[5] = {};
    float thr_f[5] = {};
    float code_inv = 1.f;       // 1 / delta of the screening codes
    uint32_t code_thr[5] = {};  // screen thresholds in code units
    float2 *d_bank = nullptr;  // nz x S, segment domain, scaled by 1/S (FFT correlator)
    float2 *d_bank_half = nullptr;  // the same for the half-bin offsets (interbin)
    void *d_gemm = nullptr;    // template matrix of the matrix correlator
    int32_t corr = 0;          // FDAS_CORR_*
    bool td = false;           // time-domain resampling search: nz trials alpha = -zmax + iz dz
    int num_cu = 256;          // compute units of the device (matrix correlator grid)
    // ws[0]: fdas_search; ws[1], ws[2]: the batched path's two slots, so that
    // a batch leaves the single-search buffers (and what the inspection,
    // interpolation and refinement calls read from them) untouched
    std::array<fdas::Workspace, 3> ws{};
    std::array<hipStream_t, 2> aux{};
    std::array<hipEvent_t, 4> events{};
    // batched path: captured per-trial launch sequence, per slot and length
    std::array<std::map<int64_t, hipGraphExec_t>, 2> graphs{};
    // persistent batch launch (one launch per up to 64 trials)
    fdas::PBatch *pbatch = nullptr;
    bool broken = false;
    // fdas_search_host: two device input buffers filled on a copy stream of
    // the plan's own; the host pointer whose copy into in_dev[staged_slot]
    // was started by the previous call (event in_ready[staged_slot])
    std::array<float *, 2> in_dev{};
    hipStream_t copy_stream = nullptr;
    std::array<hipEvent_t, 2> in_ready{};
    const float *staged_host = nullptr;
    int staged_slot = -1;
    // stage timing (fdas_plan_enable_timing)
    bool timing = false;
    std::array<hipEvent_t, FDAS_NSTAGES + 1> tev{};
    std::array<double, FDAS_NSTAGES> stage_ms{};
    int64_t timed = 0;
    // last fdas_search (not a batch or served request), for the inspection,
    // interpolation and refinement calls and the work counts
    bool searched = false;
    const float2 *last_X = nullptr;
    const double *last_med = nullptr;
    int64_t last_nb = 0;
};

namespace fdas {

extern thread_local std::string g_last_error;
void set_error(const std::string &msg);
fdas_status hip_fail(fdas_plan_s *plan, hipError_t e, const char *what);
fdas_status validate_opts(const fdas_opts &o);
void init_detection(fdas_plan_s *p, int64_t cells_plane);
fdas_status check_nsamp(int64_t nsamp, int32_t seg, int32_t h);
// Plane columns per frequency bin: 2 for a half-bin plane.
inline int cols_per_bin(const fdas_plan_s *p) { return p->opts.interbin ? 2 : 1; }
Geometry make_geometry(int64_t nsamp, int32_t S, int32_t h, int32_t W, int cpb);
int64_t series_bytes(const Geometry &g, int32_t S, int32_t nz);
int64_t candidate_bytes(const fdas_plan_s *p, const Geometry &g);
fdas_status alloc_workspace(fdas_plan_s *p, Workspace &ws, int64_t nsamp);
void destroy_workspace(Workspace &ws);
// Enqueue the whole per-series path on st.  Leaves the plan's last-search
// state alone; X_out / med_out (may be NULL) receive the normalised
// spectrum's source buffer and medians the search used (NULL for a
// time-domain plan, medians NULL for an already normalised spectrum).
// direct (may be NULL): the public records go to direct->out (at most
// direct->cap of them) and the counters to direct->count instead of
// ws.final (device aliases of page-locked host memory; FFT and matrix
// plans without refinement only).
struct DirectOut {
    fdas_cand *out;
    uint32_t cap;
    uint32_t *count;
};
fdas_status enqueue_search(fdas_plan_s *p, const Workspace &ws, const Geometry &g, int32_t in_kind,
                           const void *in_dev, float *plane, DevCand *dcands, uint32_t *dcount, hipStream_t st,
                           bool timed = false, const float2 **X_out = nullptr, const double **med_out = nullptr,
                           const DirectOut *direct = nullptr);
// Trial value of plane row iz: the drift z(iz) of a template plan, the
// acceleration trial alpha_iz of a time-domain plan.
double row_value(const fdas_plan_s *p, int32_t iz);
fdas_status accumulate_timing(fdas_plan_s *p);
// Copy a finished search's sorted candidates (count already in *ws.h_count
// after the stream reached it) into out[0..cap); sets *ncands to the true count.
fdas_status copy_candidates(const fdas_plan_s *p, const Workspace &ws, fdas_cand *out, int64_t cap,
                            int64_t *ncands, hipStream_t st);
// Plan without work buffers: options, thresholds, bank in the segment domain.
fdas_status make_plan_core(const fdas_bank_s *bank, int64_t nsamp, int32_t seg, const fdas_opts *opts,
                           fdas_plan_s **out);
fdas_status collect(fdas_plan_s *p, Workspace &ws, fdas_cand *out, int64_t cap, int64_t *ncands, hipStream_t st);

// Templates per correlation workgroup: about 13, with the number of template
// blocks rounded up to a multiple of the 8 XCDs.
inline int32_t default_tpb(int32_t nz) {
    int64_t nzb = (nz + 12) / 13;
    nzb = ((nzb + 7) / 8) * 8;
    return int32_t((nz + nzb - 1) / nzb);
}

}  // namespace fdas
