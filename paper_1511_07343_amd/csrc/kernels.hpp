// Launchers of the FDAS device kernels (gfx950).  All launches are
// asynchronous on the given stream and return the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fdas.h"

namespace fdas {

// Candidate record written by the harmonic-sum kernel (16 bytes).
struct DevCand {
    int32_t k;
    int32_t iz;
    int32_t nharm;
    float power;
};

// p[0..n) = 0 with a kernel (safe inside captured graphs).
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st);

// Batched unnormalised complex DFT of length 2^log2n (6..13), dir -1 / +1.
hipError_t launch_dft(int log2n, int dir, int64_t batch, const float2 *in, float2 *out, hipStream_t st);

// Complex DFT of z[n] = x[2n] + i x[2n+1] (M = N/2 points) into Z, natural
// order.  work: M float2 scratch (used when M > 8192).
hipError_t launch_r2c_packed(const float *x, int64_t nsamp, float2 *Z, float2 *work, hipStream_t st);

// Unpack Z into the real-input spectrum X[k], k in [0, M) (X[0] = 0), and the
// median of |X|^2 over each block of W bins (FP64 out).
hipError_t launch_unpack_median(const float2 *Z, int64_t nsamp, float2 *X, double *med, int W, hipStream_t st);

// Block medians of |X|^2 of a given spectrum.
hipError_t launch_median(const float2 *X, int64_t nb, double *med, int W, hipStream_t st);

// Segment spectra: seg s = DFT_S of Xhat[s L - h + n], n in [0, S), where
// L = (S - 2h) rounded down to a multiple of 4, Xhat = X sqrt(ln2 / m(k)) (m
// interpolated between block medians in FP64; med == nullptr means X is
// already normalised); zero outside [0, nb).
hipError_t launch_segfft(const float2 *X, const double *med, int W, int64_t nb, int log2s, int h,
                         int64_t nseg, float2 *segspec, hipStream_t st);

// Xhat = X sqrt(ln2 / m(k)) into out (inspection; the search fuses it).
hipError_t launch_normalise(const float2 *X, const double *med, int W, int64_t nb, float2 *out, hipStream_t st);

// Fused correlation: for each segment s and template iz,
//   y = IDFT_S(segspec[s] * bank[iz]) (unnormalised; bank carries 1/S),
//   plane[iz][s L + n - h] = |y[n]|^2 for n in [h, h + L), inside [0, nb),
// and beside it the screening codes of 2-bin blocks (nz x nb/2 bytes)
//   codes[iz][b] = max_{k in {2b, 2b + 1}} min(255, ceil(plane[iz][k] * code_inv)).
// With bank_half (the half-bin offsets' bank) each plane row holds 2 nb
// floats, the bins k from bank in [0, nb) and the points k + 1/2 from
// bank_half in [nb, 2 nb), and the nz x nb codes cover the pairs
// (k, k + 1/2): codes[iz][k] = max of the two points' codes.
hipError_t launch_correlate(const float2 *segspec, const float2 *bank, const float2 *bank_half, int nz, int tpb,
                            int64_t nb, int log2s, int h, int64_t nseg, float *plane, uint8_t *codes, float code_inv,
                            hipStream_t st);

// Matrix-core correlator (BF16 or FP16 operands, FP32 accumulation).
// gemm_ksteps(h): K steps of 32 (real K = 2 (2h + 1), zero padded); at most
// GM_MAX_KSTEPS (the template slice must fit the workgroup's LDS).
constexpr int GM_MAX_KSTEPS = 34;
int gemm_ksteps(int h);
// Template matrix in MFMA fragment order: gemm_bank_bytes(nz, h) bytes,
// built on the host from the FP64 taps (nz x (2h + 1) complex, tap q at
// column q + h).
size_t gemm_bank_bytes(int nz, int h);
void build_gemm_bank(const double *taps, int nz, int h, bool bf16, void *out);
// Xhat = X sqrt(ln2 / m(k)) (or X when med is NULL) as 16-bit (Re, Im) pairs.
hipError_t launch_lowp_spectrum(const float2 *X, const double *med, int W, int64_t nb, bool bf16, uint32_t *out,
                                hipStream_t st);
// plane[iz][k] = |sum_q Xhat[k - q] T_iz[q]|^2 and its block screening codes
// (as launch_correlate), over `workgroups` persistent workgroups.  nb % 4 == 0.
hipError_t launch_corr_gemm(const uint32_t *xl, int64_t nb, int h, const void *bank, int nz, bool bf16,
                            int workgroups, float *plane, uint8_t *codes, float code_inv, hipStream_t st);

// Harmonic sums over 1..nharm_max harmonics, thresholds and 3x3 local
// maxima.  codes: the 2-bin block codes written beside the plane (nz x nb/2).
// thr[i] is the threshold of 2^i harmonics, code_thr[i] (<= 0x8000) the
// screen's threshold in code units: it must not exceed the code sum of any
// bin whose exact FP32 sum reaches thr[i].  Three passes: a screen of every
// 2-bin block's bound that lists the blocks which may hold a bin reaching a
// threshold, the exact sums of their bins from the plane, and the neighbour
// test of the bins whose sums reach one.  scratch:
// harmsum_scratch_bytes(nz, nb, cell_cap, group_cap) bytes, for at most
// cell_cap listed bins in group_cap groups of 32 columns.  count[0..5] must
// start at 0: candidates are appended to cands (capacity cap) through
// count[0] (count[1] is not used), count[4] and count[5] count the listed
// bins and groups; count[2] is set to 1 if a list overflowed (the
// candidates are then incomplete).  nb (plane columns) must be a multiple of
// 32, nz at most 65535; izc < 0 sums every harmonic in the cell's own row.
// split > 0 marks a half-bin plane stored as two
// halves per row: column c (in half bins) at c / 2 for even c and at
// split + c / 2 for odd c.
size_t harmsum_scratch_bytes(int nz, int64_t nb, uint32_t cell_cap, uint32_t group_cap);
hipError_t launch_harmsum(const float *plane, const uint8_t *codes, int nz, int64_t nb, int64_t split, int izc,
                          int nharm_max,
                          const float *thr_host, const uint32_t *code_thr, void *scratch, uint32_t cell_cap,
                          uint32_t group_cap, DevCand *cands, uint32_t *count, uint32_t cap, hipStream_t st);

// min(*count, cap) records from src to dst and count[0..5] to count_dst, both
// destinations device aliases of page-locked host memory.
hipError_t launch_copy_records(const fdas_cand *src, const uint32_t *count, uint32_t cap, fdas_cand *dst,
                               uint32_t *count_dst, hipStream_t st);
// Candidate finishing: sort the first min(*count, cap) records by
// (nharm, k, iz) (k < nb plane columns, iz < nz) and write the first
// min(*count, cap, out_cap) of them as public records (r = k / (nharm cpb)
// with cpb plane columns per bin, z, FP64 significance) to out; with
// count_dst, also count[0..5] there (out and count_dst may be device aliases
// of page-locked host memory).
// scratch: cand_sort_scratch_bytes(cap) bytes.
size_t cand_sort_scratch_bytes(uint32_t cap);
hipError_t launch_finish_candidates(const DevCand *dc, const uint32_t *count, uint32_t cap, void *scratch, int nz,
                                    int64_t nb, int cpb, double zmax, double dz, fdas_cand *out, hipStream_t st,
                                    uint32_t out_cap = 0xffffffffu, uint32_t *count_dst = nullptr);

// De-dispersion: out[i][t] = sum_c fil[c][t + delays[i][c]] for t < nout
// (channel-major 8-bit filterbank, nchan x nsamp; exact integer sums stored
// as float32).  Every t + delay must lie below nsamp (the caller checks).
hipError_t launch_dedisperse(const uint8_t *fil, int nchan, int64_t nsamp, const int32_t *delays, int ndm,
                             int64_t nout, float *out, hipStream_t st);

// Time-domain resampling search: y = x resampled for drift alpha (relative
// to the mean frequency; linear interpolation, FP64 positions); normalised
// powers |X|^2 ln2 / m(k) of one trial into a plane row with their 2-bin
// codes (nb % 4 == 0); candidate drift z = alpha(iz) r with alpha(iz) =
// -alpha_max + iz 2 alpha_max / (nalpha - 1).
hipError_t launch_td_resample(const float *x, int64_t nsamp, double alpha, float *y, hipStream_t st);
hipError_t launch_td_power(const float2 *X, const double *med, int W, int64_t nb, float *row, uint8_t *qrow,
                           float code_inv, hipStream_t st);
hipError_t launch_td_drift(const uint32_t *count, uint32_t cap, double alpha_max, int nalpha, fdas_cand *cands,
                           hipStream_t st);

// Candidate refinement (Fourier interpolation off the grid): for each of the
// first min(*count, cap) public records, a pattern search over the
// fundamental (r, z) for the largest S(r, z) = sum_{j=1}^{nh} P(j r, j z),
// P the correlation power with the response evaluated at the exact offset
// and drift, starting from r = k / (nh cpb) (cpb plane columns per bin);
// levels step halvings from half a grid cell.  r, z, power and
// sigma of the records are replaced by those of the final point.  The
// spectrum is X scaled by sqrt(ln2 / m(k)) (X itself when med is NULL), as in
// the search.  A persistent grid of `workgroups` workgroups.
// Device address (on the current device) and size of the file-scope scratch
// array of the allocation-free refinement; looked up once per device.
hipError_t refine_noalloc_scratch(void **out, size_t *bytes);
hipError_t launch_refine(const float2 *X, const double *med, int W, int64_t nb, int h, int izc, double dz,
                         double zmax, int cpb, int levels, const uint32_t *count, uint32_t cap, fdas_cand *cands,
                         int workgroups, hipStream_t st);
// out[i] = S(r[i], z[i]) with nh[i] harmonics (NaN when nh[i] is not in 1..16),
// device arrays of n entries.
hipError_t launch_interp_points(const float2 *X, const double *med, int W, int64_t nb, int h, const double *r,
                                const double *z, const int32_t *nh, int64_t n, double *out, hipStream_t st);

// ------------------------------------------------ persistent batch launch
// Stages of one trial in the persistent batch kernel, in dependency order:
// segment DFTs, correlation (segment x template block), harmonic-sum screen,
// exact sums of the flagged cells, neighbour test of the hits.
enum BatchStage { BST_SEG = 0, BST_CORR = 1, BST_SCREEN = 2, BST_EXACT = 3, BST_PEAK = 4, BST_N = 5 };

// Per-trial descriptor (device memory).  X, med, seg, cnt and cands belong to
// the trial; plane, codes and hits to the ring slot it runs in.
struct BatchTrial {
    const float2 *X;
    const double *med;
    float2 *seg;
    float *plane;
    uint8_t *codes;
    void *hits;  // harmonic-sum lists, harmsum_scratch_bytes layout
    uint32_t *cnt;  // six counters, zeroed before the launch
    DevCand *cands;
    int64_t nb;
    int64_t nseg;
    uint32_t ntile[BST_N];  // tiles of each stage
    uint32_t pad;
};

// The global tile order: one packed word per tile, stage in bits 29-31,
// trial in bits 23-28, tile index within the stage in bits 0-22.
constexpr int kBatchMaxTrials = 64;
constexpr uint32_t batch_tile(uint32_t stage, uint32_t trial, uint32_t idx) {
    return (stage << 29) | (trial << 23) | idx;
}
constexpr uint32_t kBatchMaxStageTiles = 1u << 23;

// Control words: [0] next tile, [1] error flag (1: a dependency wait ran
// out, 2: a malformed tile word), [2..5] the first timed-out wait (stage,
// trial, count seen, count awaited), [6..7] unused, then done[stage][trial]
// (BST_N x ntrials tile counts).  Zeroed before the launch.
constexpr int kBatchCtlHead = 8;

// Tiles of the exact-sum and neighbour-test stages per trial.
constexpr uint32_t kBatchExactTiles = 128;
constexpr uint32_t kBatchPeakTiles = 128;
// Screen tiles: (nb / 8192 rounded up) column tiles x (nz / 8 rounded up) row bands.
uint32_t batch_screen_tiles(int64_t nb, int nz);

// The persistent kernel: `workgroups` workgroups take tiles of the global
// order from ctl[0] until it is exhausted.  A tile waits (bounded) until the
// tiles it depends on are done: correlation on the trial's segment DFTs and,
// from trial `slots` on, on the neighbour test of trial - slots (whose ring
// slot it reuses); screen on the correlation; exact sums on the screen;
// neighbour test on the exact sums.  Every dependency precedes its dependent
// in the order, so the launch cannot deadlock.  log2s 12 or 13, no half-bin
// plane.
hipError_t launch_batch_persistent(int log2s, int nharm_max, const BatchTrial *trials, int ntrials,
                                   const uint32_t *tiles, uint32_t ntiles, uint32_t *ctl, int slots,
                                   const float2 *bank, int nz, int tpb, int h, int W, int izc, float code_inv,
                                   const float *thr_host, const uint32_t *code_thr, uint32_t cell_cap,
                                   uint32_t group_cap, uint32_t cand_cap, int workgroups, hipStream_t st);
// Workgroups of the persistent kernel that fit the device at once.
hipError_t batch_persistent_workgroups(int log2s, int nharm_max, int *per_cu);

}  // namespace fdas
