/*
 * fdas.h -- C ABI of the MI355X (gfx950) Fourier Domain Acceleration Search
 * correlation hot path.
 *
 * Method: S. Dimoudi and W. Armour, "Pulsar Acceleration Searches on the GPU
 * for the Square Kilometre Array", arXiv:1511.07343.  Templates are computed
 * once in an initialisation stage and every received series then goes through
 * the per-series steps of Sec. 4: real-to-complex DFT, overlapped segments,
 * segment DFT, complex multiply-scale by every template, inverse DFT, and
 * power spectrum operations (powers with edge removal), which produce the
 * f-fdot power plane of Sec. 2 (Fig. 1).  On top of that plane this library
 * sums harmonics and reports thresholded local maxima as candidates.
 *
 * Conventions shared by every call
 *   - Every call returns an fdas_status; FDAS_OK is 0, errors are negative.
 *     fdas_last_error() gives a thread-local detail string for the last error
 *     raised on the calling thread.  No C++ exception crosses this ABI.
 *   - The caller owns every buffer it passes in; the library owns bank, plan
 *     and server objects and frees them in the matching *_destroy call.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  hip_stream arguments are a
 *     hipStream_t passed as void* (NULL = the default stream).
 *   - Complex data is interleaved (re, im) float32 ("c64") unless stated.
 *   - Series length N is a power of two in [2^10, 2^26]; the spectrum has
 *     Nb = N/2 bins, bin 0 (DC) is zeroed and the Nyquist bin dropped.
 *   - The f-fdot plane is float32[nz][Nb], template-major (row iz holds all
 *     Nb frequency bins of template iz, contiguous in k); with
 *     fdas_opts.interbin it is float32[nz][2 Nb], row iz holding bins
 *     k = 0 .. Nb-1 in its first Nb floats and the points k + 1/2 between
 *     bins k and k + 1 in the next Nb.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fdas_status {
    FDAS_OK = 0,
    FDAS_E_INVAL = -1,    /* an argument is out of range or inconsistent          */
    FDAS_E_NOMEM = -2,    /* device or host allocation failed / budget exceeded   */
    FDAS_E_DEVICE = -3,   /* a HIP call failed; the plan is unusable afterwards   */
    FDAS_E_OVERFLOW = -4, /* more candidates than capacity; *ncands = true count  */
    FDAS_E_BUSY = -5,     /* server queue full                                    */
    FDAS_E_TIMEOUT = -6   /* fdas_poll: nothing completed within the timeout      */
} fdas_status;

typedef struct fdas_bank_s fdas_bank;
typedef struct fdas_plan_s fdas_plan_t;
typedef struct fdas_server_s fdas_server;

/* One candidate: a thresholded local maximum of an nharm-harmonic sum whose
 * top harmonic sits at plane cell (iz, k).  r and z describe the fundamental:
 * r = k / nharm bins, z = z(iz) / nharm bins with z(iz) = -zmax + iz * dz
 * (with fdas_opts.interbin, k counts half bins and r = k / (2 nharm)).
 * power is the harmonic sum; sigma its Gaussian-equivalent single-trial
 * significance (FP64 on the host). 40 bytes. */
typedef struct fdas_cand {
    int64_t k;
    int32_t iz;
    int32_t nharm;
    double r;
    double z;
    float power;
    float sigma;
} fdas_cand;

/* Input kinds for fdas_search. */
enum {
    FDAS_IN_SERIES_F32 = 0,              /* float32[N] time series                    */
    FDAS_IN_SPECTRUM_C64 = 1,            /* c64[Nb] raw spectrum; library normalises  */
    FDAS_IN_SPECTRUM_C64_NORMALISED = 2  /* c64[Nb] already normalised spectrum       */
};

/* Search options.  Zero-initialise and call fdas_default_opts() first. */
typedef struct fdas_opts {
    double sigma;                /* detection threshold, single-trial sigma (default 6)      */
    int32_t nharm_max;           /* 1, 2, 4, 8 or 16 harmonics summed (default 16)           */
    int32_t median_window;       /* normalisation block length W, 32..8192, pow2 (def. 1024) */
    int64_t cand_capacity;       /* device candidate buffer entries (default 1<<20)          */
    int32_t templates_per_block; /* templates per correlation workgroup, 0 = automatic       */
    int32_t correlator;          /* FDAS_CORR_FFT_F32 (default) or a matrix form, see below   */
    int32_t refine_levels;       /* candidate refinement levels, 0 = off (default), <= 20     */
    int32_t interbin;            /* 1 = half-bin plane (2 Nb columns), 0 = off (default)      */
    int32_t batch_launch;        /* fdas_search_batch: FDAS_BATCH_STREAMS (default) or        */
                                 /* FDAS_BATCH_PERSISTENT, see fdas_search_batch              */
} fdas_opts;
enum { FDAS_BATCH_STREAMS = 0, FDAS_BATCH_PERSISTENT = 1 };

/* Half-bin plane (interbin = 1), an extension past the paper's method: a
 * second template bank at offsets q + 1/2, T'_z[q] = conj(A(q + 1/2, z)) /
 * norm for q = -h .. h-1 (the 2h offsets within h of the half-bin point),
 * gives P(k + 1/2, z) (the interpolated power of the refinement note below
 * at r = k + 1/2), stored beside P(k, z) (see the plane layout above).  The
 * harmonic sums, thresholds and peaks then run on the half-bin grid, point
 * c = 2k or 2k + 1 for r = c / 2, with candidate k = c, so a tone between
 * two bins keeps at least sinc^2(1/4) = 0.81 of its power on the grid
 * instead of sinc^2(1/2) = 0.41.  Twice the correlation
 * work and plane memory.  FFT correlator only (INVAL with a matrix one). */

/* Candidate refinement (refine_levels > 0), an extension past the paper's
 * method: Fourier interpolation of the correlation at fractional frequency
 * and drift.  The response A(q, z) of Sec. 2 is evaluated at the exact
 * offsets r - k of the bins k with |r - k| <= h, so that
 *   P(r, z) = |sum_k Xhat[k] conj(A(r - k, z))|^2 / sum_k |A(r - k, z)|^2
 * (Xhat zero outside [0, Nb)); at integer r and a bank z it is the plane
 * cell.  S(r, z) = sum_{j=1}^{nharm} P(j r, j z) sums the harmonics at their
 * exact positions.  Each candidate's fundamental then moves by a pattern
 * search: from r = k / nharm (k / (2 nharm) with interbin),
 * z = ((iz - izc) dz) / nharm (izc = zmax / dz),
 * level l = 1 .. refine_levels looks at the 8 neighbours at steps
 * (2^-l / nharm, dz 2^-l / nharm), z offset major then r offset, each -1, 0,
 * +1, and moves to the first that beats every earlier value of the level,
 * the centre's included; a neighbour with |nharm z| > zmax is skipped.  The
 * record's r, z, power (= S) and sigma (of S, nharm harmonics) describe the
 * final point; k, iz and nharm still name the plane cell found.  FP64, on
 * the device, before the records are copied; its time is stage 5 of the
 * stage timers. */

/* Correlator of a plan.  FDAS_CORR_FFT_F32: overlap-save segments, FP32 DFTs
 * (Sec. 2, Sec. 4 steps 3-7).  FDAS_CORR_GEMM_BF16 / FDAS_CORR_GEMM_F16:
 * Eq. (1) summed directly as one real matrix product on the matrix cores
 * with BF16 / FP16 operands (spectrum and taps rounded to nearest) and FP32
 * accumulation; the segment length is then unused, and the half-width h must
 * be at most 271 (zmax <= 510) or fdas_plan returns INVAL.  A precision
 * variant: its powers carry the 16-bit rounding of the operands. */
enum { FDAS_CORR_FFT_F32 = 0, FDAS_CORR_GEMM_BF16 = 1, FDAS_CORR_GEMM_F16 = 2 };

void fdas_default_opts(fdas_opts *opts);

/* ---------------------------------------------------------------- templates
 * Sec. 2: one inverse-filter template per drift trial z = -zmax + iz * dz,
 * iz = 0 .. 2 zmax / dz.  Template taps are the conjugate of the Fourier
 * response A(q, z) of a tone drifting by z bins, q = -h .. h, normalised to
 * unit energy, computed in FP64 from the Fresnel-integral closed form.
 * h = ceil(zmax / 2) + 16.  Host-only: no device memory is touched.
 * Errors: FDAS_E_INVAL unless 0 <= zmax <= 1200, dz > 0, 2 zmax / dz an
 * integer (to 1e-9) and the bank has at most 4801 templates. */
fdas_status fdas_make_templates(double zmax, double dz, fdas_bank **out);
int32_t fdas_bank_nz(const fdas_bank *bank);
int32_t fdas_bank_halfwidth(const fdas_bank *bank);
double fdas_bank_z(const fdas_bank *bank, int32_t iz);
/* Copy template iz's 2h+1 taps (q = -h..h) as interleaved FP64 (re, im) into
 * re_im_out[2 * (2h + 1)] (host).  FDAS_E_INVAL for a bad iz. */
fdas_status fdas_bank_taps(const fdas_bank *bank, int32_t iz, double *re_im_out);
void fdas_bank_destroy(fdas_bank *bank);

/* ------------------------------------------------------------ significance
 * Threshold reading of "n-sigma": thr solves Q(nharm, thr) = Phi_c(sigma),
 * where Q(n, S) = exp(-S) sum_{i<n} S^i / i! is the survival function of a
 * sum of n unit-mean exponential powers and Phi_c the Gaussian upper tail.
 * fdas_significance inverts it.  Host-only, FP64. */
fdas_status fdas_threshold(double sigma, int32_t nharm, double *thr);
fdas_status fdas_significance(double power, int32_t nharm, double *sigma);

/* -------------------------------------------------------------------- plan
 * Per-series state for one (bank, nsamp, seg): the bank transformed to the
 * segment domain (c64[nz][seg], each template wrapped circularly, DFT'd in
 * FP64 and scaled by 1/seg -- the "scale" of the multiply step), and every
 * device work buffer, allocated once.  seg is the overlap-save segment length
 * (Sec. 2, Sec. 4 steps 3-6): a power of two in [256, 8192], >= 4h; each
 * segment yields seg - 2h valid bins, of which the first (seg - 2h) rounded
 * down to a multiple of 4 are kept (the rest come from the next segment).
 * Needs a visible GPU (it allocates).
 * Errors: INVAL (nsamp, seg, opts), NOMEM, DEVICE.  A plan is not
 * thread-safe; calls on it are ordered on the stream they are given. */
fdas_status fdas_plan(const fdas_bank *bank, int64_t nsamp, int32_t seg,
                      const fdas_opts *opts, fdas_plan_t **out);
/* Time-domain resampling search (the other acceleration search named in
 * Sec. 1): a plan of nalpha acceleration trials alpha_i = -alpha_max + i d,
 * d = 2 alpha_max / (nalpha - 1) (alpha = 0 when nalpha is 1), where alpha
 * is the frequency drift over the observation relative to the mean
 * frequency (a tone of mean frequency r bins drifts by z = alpha r bins).
 * fdas_search on this plan (float32 series input only) resamples the series
 * for each trial onto the axis tau = v + alpha v^2 / 2 (v the time from the
 * middle of the observation, in units of its length; linear interpolation,
 * zero outside the series), takes its real DFT and block-median
 * normalisation as in the template search, writes the powers as plane row i
 * (plane_dev: float32[nalpha][Nb]), and sums harmonics along each row (all
 * harmonics of a trial lie in its own spectrum) before the same thresholds
 * and 3x3 peaks.  Candidates: iz is the trial, r = k / nharm the
 * fundamental's mean frequency, z = alpha_iz r its drift.  One long DFT per
 * trial: the expensive method the correlation search replaces.  opts:
 * sigma, nharm_max, median_window and cand_capacity apply; correlator,
 * interbin and refine_levels must be left at their defaults (INVAL
 * otherwise).  INVAL unless 1 <= nalpha <= 4801 and 0 <= alpha_max <= 0.5.
 * fdas_search_batch, fdas_refine and fdas_interp_power return INVAL on such a
 * plan. */
fdas_status fdas_td_plan(int64_t nsamp, double alpha_max, int32_t nalpha, const fdas_opts *opts,
                         fdas_plan_t **out);
int64_t fdas_plan_nbins(const fdas_plan_t *plan);
/* Rows of the plan's plane (templates, or acceleration trials of a
 * time-domain plan) and the trial value of row iz: z(iz) = -zmax + iz dz bins
 * for a template plan (Sec. 2), alpha_iz as defined with fdas_td_plan for a
 * time-domain plan.  NaN for a NULL plan or iz outside [0, rows). */
int32_t fdas_plan_rows(const fdas_plan_t *plan);
double fdas_plan_row_value(const fdas_plan_t *plan, int32_t iz);
int64_t fdas_plan_device_bytes(const fdas_plan_t *plan);
void fdas_plan_destroy(fdas_plan_t *plan);

/* One series through the whole hot path (Sec. 4 steps 2-7, then harmonic sum
 * and peaks):
 *   in_kind/in_dev  device input: float32[nsamp] series, or c64[Nb] spectrum
 *                   (caller-owned, read-only).
 *   plane_dev       NULL, or device float32[nz][Nb] (float32[nz][2 Nb] with
 *                   interbin) that receives the plane (16-byte aligned, else
 *                   INVAL).
 *   cands_host      host array of cap entries; receives candidates sorted by
 *                   (nharm, k, iz).  May be NULL when cap is 0.
 *   ncands          receives the number of candidates found.
 *   hip_stream      stream the work is ordered on; the call returns after the
 *                   candidates are on the host (the plane, if requested, is
 *                   complete when the stream is).
 * Errors: INVAL, DEVICE, OVERFLOW (cap or cand_capacity too small: the first
 * min(cap, found) candidates in sorted order of those captured are returned
 * and *ncands holds the true count; also when the internal list of bins
 * that may reach a threshold overflowed (4 x cand_capacity bins in
 * 2 x cand_capacity groups of 32 columns; with the automatic capacity, at
 * least every bin of planes up to 2^24 bins), in which case the candidates
 * are incomplete and *ncands is a lower bound). */
fdas_status fdas_search(fdas_plan_t *plan, int32_t in_kind, const void *in_dev,
                        float *plane_dev, fdas_cand *cands_host, int64_t cap,
                        int64_t *ncands, void *hip_stream);

/* One float32 series of nsamp samples in host memory through the same path
 * as fdas_search with FDAS_IN_SERIES_F32, the host-to-device transfer of
 * Sec. 4 step 1 included and overlapped as that step allows: the plan keeps
 * two device input buffers (8 nsamp bytes, allocated on the first call) and a
 * copy stream of its own.
 *   series_host  the series to search now.  If the previous call on this plan
 *                named the same pointer as its next_host, its copy has been
 *                running since then and is waited for; otherwise it is copied
 *                on hip_stream first.
 *   next_host    NULL, or the series the caller will pass to the next call:
 *                its copy into the other input buffer starts now on the copy
 *                stream, overlapping this search.  The caller must keep that
 *                memory unchanged until the next call returns.  With
 *                page-locked memory (hipHostMalloc) the copy runs
 *                asynchronously; with pageable memory it is still correct but
 *                may not overlap.
 * Other arguments, outputs, errors and the return point (candidates on the
 * host) are those of fdas_search.  INVAL for a NULL series_host. */
fdas_status fdas_search_host(fdas_plan_t *plan, const float *series_host, const float *next_host,
                             float *plane_dev, fdas_cand *cands_host, int64_t cap, int64_t *ncands,
                             void *hip_stream);

/* Stage timing (measurement hook).  While enabled, fdas_search records a HIP
 * event pair around each stage on the stream the stage runs on and adds the
 * elapsed times (ms) into per-stage totals: 0 real-input DFT, 1 unpack and
 * block medians, 2 segment DFTs, 3 fused multiply / inverse DFT / power,
 * 4 harmonic sum, peaks and candidate ordering, 5 candidate refinement
 * (zero when off).  fdas_plan_stage_times copies the FDAS_NSTAGES
 * totals and the number of searches timed; enabling resets them. */
#define FDAS_NSTAGES 6
fdas_status fdas_plan_enable_timing(fdas_plan_t *plan, int32_t enable);
fdas_status fdas_plan_stage_times(const fdas_plan_t *plan, double *ms_out, int64_t *nsearch_out);

/* Work counts of the last fdas_search on this plan (diagnostics): out3[0]
 * candidates found, out3[1] plane cells the harmonic-sum screen passed on to
 * the exact FP32 sums, out3[2] groups of 32 columns holding those cells.
 * INVAL if no search has completed on the plan. */
fdas_status fdas_plan_search_counts(const fdas_plan_t *plan, int64_t *out3);

/* Several float32 series, possibly of different power-of-two lengths
 * nsamp[i] <= the plan's nsamp, through the hot path (no plane is returned).
 * The work is ordered after what hip_stream holds when the call is made, and
 * hip_stream is ordered after it on return.
 * With opts.batch_launch FDAS_BATCH_STREAMS (the default), and for plans the
 * persistent form does not cover: consecutive trials alternate between two
 * library-owned streams and two work buffers, so that one trial's harmonic
 * sums overlap the next trial's correlation, each trial's launches captured
 * once per length in a HIP graph; every kernel runs at its own occupancy.
 * With FDAS_BATCH_PERSISTENT, the FFT correlator, segment length 4096 or
 * 8192 and no half-bin plane,
 * up to 64 trials at a time go through ONE launch of a persistent kernel (a
 * longer batch takes one launch per 64): per trial the real DFT and block
 * medians run first, then the persistent workgroups take tiles from a device
 * work queue -- segment DFTs, correlation tiles (segment x template block),
 * harmonic-sum screen, exact-sum and neighbour-test tiles -- each trial's
 * next stage released by a per-trial completion counter, with consecutive
 * trials' stages interleaved (Sec. 1: an observation yields thousands of
 * independent series; Sec. 4 steps 2-7 for each).  The clears, front end,
 * persistent launch and count copies are captured in one HIP graph per call;
 * candidates are sorted per trial afterwards.  Device memory, allocated on
 * the first such call and kept by the plan: per trial (up to 64) its
 * spectrum, medians, segment spectra and candidate records; four plane /
 * screening-code / list slots shared round-robin by the trials.  On MI355X
 * the persistent form is the slower one (about 0.6 x the two-stream rate at
 * 2^23 samples): its memory-bound harmonic-sum tiles run at the correlation
 * tiles' occupancy of two workgroups per compute unit, which the separate
 * kernels of the two-stream form do not share.
 * Either way a batch leaves the buffers of fdas_search alone: the
 * inspection, interpolation, refinement and work-count calls keep describing
 * the plan's last fdas_search.  Trial i's candidates go to
 * cands_host + sum_{j<i} cap[j], count to ncands[i].  Returns the first error,
 * or OVERFLOW if any trial overflowed; DEVICE if a dependency wait inside the
 * persistent kernel ran out (the plan is then unusable). */
fdas_status fdas_search_batch(fdas_plan_t *plan, int32_t n, const float *const *series_dev,
                              const int64_t *nsamp, fdas_cand *cands_host, const int64_t *cap,
                              int64_t *ncands, void *hip_stream);

/* Autotuner for many-trial use: times the segment DFTs plus the fused
 * correlation for every segment length in {1024, 2048, 4096, 8192} that is
 * >= 4h and templates per workgroup in {7, 13, 26}, on a seeded synthetic
 * noise series of nsamp samples, and returns the fastest (seg, templates per
 * block) and its time in ms.  With opts->batch_launch =
 * FDAS_BATCH_PERSISTENT the lengths are {4096, 8192} (those of the
 * persistent launch) and the time is the persistent batch's wall time per
 * trial over 8 copies of the series.  cache_path (may be NULL) names a text file of earlier
 * results keyed by (GPU arch, nsamp, nz, h, lengths tried); a hit skips the measurement, a
 * miss appends the new result.  Needs a GPU; allocates temporary plans. */
fdas_status fdas_autotune(const fdas_bank *bank, int64_t nsamp, const fdas_opts *opts,
                          const char *cache_path, int32_t *seg_out, int32_t *tpb_out, double *ms_out);

/* Fourier-interpolated harmonic sums S(r[i], z[i]) with nharm[i] harmonics
 * (1..16; NaN otherwise) on the normalised spectrum of the plan's last
 * fdas_search (the definition is given with refine_levels above), for n
 * points given in host arrays; results to power_out[n] (host).  For input
 * kind FDAS_IN_SPECTRUM_C64_NORMALISED the caller's spectrum buffer must
 * still hold that spectrum.  Synchronous; allocates 28 n bytes of device
 * memory for the call.  INVAL if no search has completed on the plan or
 * n < 0; NOMEM if the buffers cannot be allocated. */
fdas_status fdas_interp_power(fdas_plan_t *plan, int64_t n, const double *r, const double *z, const int32_t *nharm,
                              double *power_out, void *hip_stream);

/* Refine chosen candidate records, in place, on the normalised spectrum of
 * the plan's last fdas_search: the pattern search described with
 * refine_levels above, with `levels` levels (1..20), applied to
 * cands[0..n) (host records as fdas_search returned them; k, iz and nharm
 * are read, r, z, power and sigma replaced).  For callers that refine only
 * the candidates they keep (e.g. the most significant after sifting)
 * rather than every record of the search.  For input kind
 * FDAS_IN_SPECTRUM_C64_NORMALISED the caller's spectrum buffer must still
 * hold that spectrum.  Synchronous; allocates 40 n + 4 bytes of device
 * memory for the call.  INVAL if no search has completed on the plan, n < 0,
 * levels out of range or a record's nharm is not 1, 2, 4, 8 or 16; NOMEM if
 * the buffer cannot be allocated. */
fdas_status fdas_refine(fdas_plan_t *plan, fdas_cand *cands, int64_t n, int32_t levels, void *hip_stream);

/* fdas_refine without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, refinement and results as
 * fdas_refine (bit-identical: the same kernels), but the records and their
 * count are staged in a fixed device array that the library holds for the
 * life of the process, FDAS_REFINE_NOALLOC_MAX records large (one array per
 * GPU), instead of a per-call allocation; nothing is allocated or freed.
 * INVAL when n > FDAS_REFINE_NOALLOC_MAX or when the current device is not
 * the plan's, besides fdas_refine's own INVAL cases.  Every call on one GPU
 * uses that GPU's one array: calls that overlap on a GPU (from several
 * threads, or on several streams without ordering) race and must be
 * serialised by the caller.  Synchronous.  For the copies to be capturable
 * and asynchronous, cands should be page-locked host memory. */
#define FDAS_REFINE_NOALLOC_MAX 16384
fdas_status fdas_refine_noalloc(fdas_plan_t *plan, fdas_cand *cands, int64_t n, int32_t levels,
                                void *hip_stream);

/* Test hook: copy the last search's normalised spectrum (c64[Nb]) and block
 * medians (double[ceil(Nb/W)]) to device buffers; either pointer may be NULL. */
fdas_status fdas_plan_fetch_spectrum(fdas_plan_t *plan, void *spectrum_dev, double *medians_dev,
                                     void *hip_stream);

/* De-dispersion, the step that produces the series (Sec. 1: one series per
 * dispersion-measure trial, ~6000 for an SKA beam).  fil_dev: device
 * channel-major 8-bit filterbank (4-byte aligned), nchan rows of nsamp
 * samples, channel c at
 * f_top - c foff MHz (foff >= 0: descending frequencies).  Trial i shifts
 * channel c by d[i][c] = floor(k DM_i (f_c^-2 - f_top^-2) / tsamp + 1/2) samples
 * (k = 4.148808e3 s MHz^2 pc^-1 cm^3, the cold-plasma dispersion delay,
 * rounded to the nearest sample; tsamp in s; dms: host array of ndm values
 * >= 0, pc cm^-3) and writes out_dev[i][t] = sum_c fil[c][t + d[i][c]] for
 * t < nout (device float32[ndm][nout]; exact integer sums).  INVAL unless
 * nout <= nsamp - max d, every delay < 2^31, 1 <= nchan, ndm <= 65536 and
 * every frequency is positive.  Synchronous; allocates 4 ndm nchan bytes of device memory for
 * the call.  The output rows are series for fdas_search (nout a power of
 * two) or fdas_search_batch. */
fdas_status fdas_dedisperse(const uint8_t *fil_dev, int32_t nchan, int64_t nsamp, double f_top, double foff,
                            double tsamp, const double *dms, int32_t ndm, int64_t nout, float *out_dev,
                            void *hip_stream);

/* Batched unnormalised complex DFT of length 2^log2n (6 <= log2n <= 13) on
 * device c64 data, in-place allowed: out[b][f] = sum_n in[b][n] e^{-+2 pi i n f / 2^log2n},
 * sign - for inverse = 0, + for inverse = 1.  The workgroup DFT of the hot path. */
fdas_status fdas_dft_c64(int32_t log2n, int32_t inverse, int64_t batch, const void *in_dev,
                         void *out_dev, void *hip_stream);

/* ------------------------------------------------------------------ server
 * Continuous-batching request loop on one GPU.  The bank and per-length
 * plans stay resident; requests (float32 host series, power-of-two lengths
 * up to max_nsamp) are copied on submit, admitted while a slot is free and
 * their device bytes fit -- within hbm_budget bytes of work buffers, or, with
 * hbm_budget 0, within the device's free HBM read (hipMemGetInfo) at the
 * moment a new work buffer is needed, less a reserve of 512 MiB + 1% of the
 * total -- and run concurrently, one stream per slot.  Work buffers are
 * cached per length and reused; idle ones of other lengths are freed when a
 * request does not fit.  A finished request's records are copied
 * asynchronously into a page-locked buffer of the server's pool, so the
 * scheduler never waits on a copy.  Each result is what fdas_search returns
 * for the same series alone.  NOMEM if one request of max_nsamp does not fit
 * the budget (or the free HBM) at creation. */
fdas_status fdas_server_create(const fdas_bank *bank, int32_t seg, const fdas_opts *opts,
                               int64_t max_nsamp, size_t hbm_budget, int32_t max_slots,
                               fdas_server **out);
/* Non-blocking; FDAS_E_BUSY if the pending queue holds 65536 requests. */
fdas_status fdas_submit(fdas_server *server, const float *series_host, int64_t nsamp,
                        uint64_t tag);
/* Wait up to timeout_ms (< 0 = forever) for a completed request; fill its tag,
 * candidates (sorted as fdas_search), count, and latency (submit -> result
 * ready, seconds).  FDAS_E_TIMEOUT if none completed; a completed request's
 * own error (e.g. OVERFLOW) is returned with its tag filled in. */
fdas_status fdas_poll(fdas_server *server, uint64_t *tag, fdas_cand *cands, int64_t cap,
                      int64_t *ncands, double *latency_s, int32_t timeout_ms);
/* Requests submitted but not yet polled. */
int64_t fdas_server_outstanding(const fdas_server *server);
void fdas_server_destroy(fdas_server *server);

/* --------------------------------------------------------------- errors */
const char *fdas_strerror(fdas_status status);
const char *fdas_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDAS_H */
