// FDAS device kernels for gfx950 (CDNA4).  Steps follow Sec. 4 of Dimoudi &
// Armour (arXiv:1511.07343): real-to-complex DFT (step 2), overlapped segments
// and their DFTs (steps 3-4, the overlap copy folded into the segment loader),
// complex multiply-scale by every template (step 5), inverse DFT (step 6) and
// power with edge removal (step 7) fused into one kernel; then harmonic sums,
// thresholds and local maxima on the resulting f-fdot plane.
#include "device_common.hpp"
#include "fft_wg.hpp"
#include "kernels.hpp"

#include <cmath>

namespace fdas {

namespace {

// Threads per workgroup for a transform of 2^log2s points.
constexpr int fft_threads(int log2s) {
    return log2s >= 12 ? 256 : log2s == 11 ? 128 : log2s >= 8 ? 64 : 32;
}

// Threads per workgroup of the fused correlation kernel, and the waves per
// SIMD its register budget is held to (4096 points on the integer grid fit
// 128 registers).
constexpr int corr_threads(int log2s) { return fft_threads(log2s); }
constexpr int corr_waves(int log2s, bool interbin) { return log2s == 12 && !interbin ? 4 : 2; }
// Whether the fused correlation kernel holds its segment's spectrum in
// registers across the templates of its block (the persistent kernel's
// correlation tiles always do): at 8192 points (218 VGPRs,
// still two waves per SIMD) and 2048 (139 VGPRs, three waves instead of
// four, yet faster); not at 4096, whose 128-register budget would spill, nor
// for the half-bin plane, which measured slower.
constexpr bool corr_hold(int log2s, bool interbin) { return (log2s == 13 || log2s == 11) && !interbin; }

// 8 XCDs on MI355X; workgroups are dispatched to XCDs round-robin by index.
constexpr int kXcds = 8;

// Plane stores bypass the L2 retention (streaming), so that they do not evict
// the templates an XCD reuses across segments.
typedef float f32x4v __attribute__((ext_vector_type(4)));

// Raw buffer access (gfx950 buffer instructions): a resource with a 64-bit
// base and a byte extent, a 32-bit lane offset and a wave-uniform constant
// offset.  Accesses past the extent read 0 / are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), short(0), bytes, 0x00020000);
}
// element (lane + k) of a float2 array
__device__ __forceinline__ float2 buffer_load_f2(__amdgpu_buffer_rsrc_t r, int lane, int k) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, lane * 8, k * 8, 0));
}
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
constexpr int kCachePolicyNT = 2;  // non-temporal (streaming) store
__device__ __forceinline__ void buffer_store_nt_f4(float4 v, __amdgpu_buffer_rsrc_t r, int byte_off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4v, v), r, byte_off, 0, kCachePolicyNT);
}
__device__ __forceinline__ void buffer_store_nt_u16(uint16_t v, __amdgpu_buffer_rsrc_t r, int byte_off) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, byte_off, 0, kCachePolicyNT);
}

// Valid points per segment: S - 2h rounded down to a multiple of 4, so that
// the correlation's 4-bin store chunks (and the 2-bin blocks of the screening
// codes) never straddle two segments.
__host__ __device__ constexpr int64_t seg_valid(int S, int h) { return int64_t((S - 2 * h) & ~3); }

// ------------------------------------------------------------- plain DFT
template <int LOG2S, int DIR>
__global__ __launch_bounds__(fft_threads(LOG2S)) void k_dft(const float2 *__restrict__ in,
                                                            float2 *__restrict__ out) {
    using Sh = FftShape<LOG2S, fft_threads(LOG2S)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * Sh::S;
    Twiddles<Sh, DIR> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = in[base + t + Sh::NT * m];
    fft_wg<Sh, DIR>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) out[base + t + Sh::NT * m] = v[m];
}

// ------------------------------------------------------- real input DFT
// z[n] = x[2n] + i x[2n+1] is read as float2 directly from the series.

// M = 2^LOG2M <= 8192: one workgroup.
template <int LOG2M>
__global__ __launch_bounds__(fft_threads(LOG2M)) void k_r2c_small(const float2 *__restrict__ z,
                                                                  float2 *__restrict__ Z) {
    using Sh = FftShape<LOG2M, fft_threads(LOG2M)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = z[t + Sh::NT * m];
    fft_wg<Sh, -1>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) Z[t + Sh::NT * m] = v[m];
}

// Workgroup i of n: with n a multiple of the 8 XCDs, the index that puts a
// contiguous range of n / 8 columns (or rows) on each XCD, so that the
// neighbours whose strided accesses share cache lines share its L2.
__device__ __forceinline__ int64_t xcd_spread(int64_t i, int64_t n) {
    return (n % kXcds == 0) ? (i % kXcds) * (n / kXcds) + i / kXcds : i;
}

// Four-step M = M1 * M2 (n = n2 + M2 n1, k = k1 + M1 k2).
// Pass A, one workgroup per column n2: DFT over n1, times exp(-2 pi i n2 k1 / M),
// stored at work[n2 + M2 k1].
template <int LOG2M1>
__global__ __launch_bounds__(fft_threads(LOG2M1)) void k_r2c_cols(const float2 *__restrict__ z,
                                                                  float2 *__restrict__ work,
                                                                  int log2m2) {
    using Sh = FftShape<LOG2M1, fft_threads(LOG2M1)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    const int64_t M2 = int64_t(1) << log2m2;
    const int64_t M = M2 << LOG2M1;
    const int64_t n2 = xcd_spread(blockIdx.x, gridDim.x);  // adjacent columns share lines
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = z[n2 + M2 * (t + Sh::NT * m)];
    fft_wg<Sh, -1>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) {
        const int64_t k1 = t + Sh::NT * m;
        const int64_t idx = (n2 * k1) & (M - 1);
        double s, c;
        sincospi(-2.0 * double(idx) / double(M), &s, &c);
        const float2 w = make_float2(float(c), float(s));
        work[n2 + M2 * k1] = cmul(v[m], w);
    }
}

// Pass B, one workgroup per row k1: DFT over n2 -> Z[k1 + M1 k2].
template <int LOG2M2>
__global__ __launch_bounds__(fft_threads(LOG2M2)) void k_r2c_rows(const float2 *__restrict__ work,
                                                                  float2 *__restrict__ Z,
                                                                  int log2m1) {
    using Sh = FftShape<LOG2M2, fft_threads(LOG2M2)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    const int64_t k1 = xcd_spread(blockIdx.x, gridDim.x);  // adjacent rows' outputs share lines
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = work[(k1 << LOG2M2) + t + Sh::NT * m];
    fft_wg<Sh, -1>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) Z[k1 + (int64_t(t + Sh::NT * m) << log2m1)] = v[m];
}

// The same two passes with four columns (rows) per workgroup, column c
// transformed by the threads t with t mod 4 = c (for 2^7 to 2^11 points): a
// wave's load or store of one register then covers 16 rows of four adjacent
// columns, 32 contiguous bytes each, instead of 64 rows of one column.  Each
// column's LDS region is offset by 16 banks from the previous.
constexpr int kR2cGroup = 4;

template <class Sh>
constexpr int r2c_region() {
    return Sh::LDS_FLOAT2 + 8;
}

template <int LOG2M1>
__global__ __launch_bounds__(fft_threads(LOG2M1) * kR2cGroup) void k_r2c_cols4(const float2 *__restrict__ z,
                                                                                float2 *__restrict__ work,
                                                                                int log2m2) {
    using Sh = FftShape<LOG2M1, fft_threads(LOG2M1)>;
    __shared__ float2 lds[kR2cGroup * r2c_region<Sh>()];
    const int c = threadIdx.x & (kR2cGroup - 1);
    const int t = threadIdx.x / kR2cGroup;
    const int64_t M2 = int64_t(1) << log2m2;
    const int64_t M = M2 << LOG2M1;
    const int64_t n2 = xcd_spread(blockIdx.x, gridDim.x) * kR2cGroup + c;  // adjacent groups share lines
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = z[n2 + M2 * (t + Sh::NT * m)];
    fft_wg<Sh, -1>(v, lds + c * r2c_region<Sh>(), tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) {
        const int64_t k1 = t + Sh::NT * m;
        const int64_t idx = (n2 * k1) & (M - 1);
        double s, co;
        sincospi(-2.0 * double(idx) / double(M), &s, &co);
        const float2 w = make_float2(float(co), float(s));
        work[n2 + M2 * k1] = cmul(v[m], w);
    }
}

template <int LOG2M2>
__global__ __launch_bounds__(fft_threads(LOG2M2) * kR2cGroup) void k_r2c_rows4(const float2 *__restrict__ work,
                                                                                float2 *__restrict__ Z,
                                                                                int log2m1) {
    using Sh = FftShape<LOG2M2, fft_threads(LOG2M2)>;
    __shared__ float2 lds[kR2cGroup * r2c_region<Sh>()];
    const int c = threadIdx.x & (kR2cGroup - 1);
    const int t = threadIdx.x / kR2cGroup;
    const int64_t k1 = xcd_spread(blockIdx.x, gridDim.x) * kR2cGroup + c;
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = work[(k1 << LOG2M2) + t + Sh::NT * m];
    fft_wg<Sh, -1>(v, lds + c * r2c_region<Sh>(), tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) Z[k1 + (int64_t(t + Sh::NT * m) << log2m1)] = v[m];
}

// ------------------------------------------------------ medians of |X|^2
// Order statistics of W powers in LDS by radix selection on their bit
// patterns (non-negative floats and +inf order as their unsigned bits): four
// passes of 8 bits, each a 256-bucket histogram and a scan that finds the
// bucket holding the wanted rank.  The result is the exact rank-r value, as
// a sort would give.
constexpr int kMedThreads = 256;

static_assert(kMedThreads == 256, "one histogram bucket per thread");

struct SelectScratch {
    uint32_t hist[256];
    uint32_t wave_tot[kMedThreads / 64];
    uint32_t pick[2];  // bucket, rank within it
};

__device__ uint32_t select_rank(const uint32_t *u, int n, uint32_t rank, SelectScratch &sc) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        sc.hist[t] = 0;  // kMedThreads == 256 buckets
        __syncthreads();
        for (int i = t; i < n; i += kMedThreads) {
            const uint32_t key = u[i];
            if ((key & mask) == prefix) atomicAdd(&sc.hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        // inclusive scan of the 256 counts: within each wave, then across the 4
        const uint32_t c = sc.hist[t];
        uint32_t incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) sc.wave_tot[wave] = incl;
        __syncthreads();
        for (int w = 0; w < wave; ++w) incl += sc.wave_tot[w];
        const uint32_t excl = incl - c;
        if (excl <= rank && rank < incl) {
            sc.pick[0] = uint32_t(t);
            sc.pick[1] = rank - excl;
        }
        __syncthreads();
        prefix |= sc.pick[0] << shift;
        mask |= 255u << shift;
        rank = sc.pick[1];
        __syncthreads();  // pick and hist are rewritten by the next pass
    }
    return prefix;
}

// Median of the n valid keys (mean of the middle pair for even n), in FP64:
// rank (n - 1) / 2 by selection; for even n the next rank is that value again
// when it occurs more than once up to it, else the smallest larger key.
__device__ double median_select(const uint32_t *u, int n, SelectScratch &sc) {
    const uint32_t r1 = uint32_t(n - 1) >> 1;
    const uint32_t v1 = select_rank(u, n, r1, sc);
    if (n & 1) return double(__uint_as_float(v1));
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t le = 0, above = 0xffffffffu;
    for (int i = t; i < n; i += kMedThreads) {
        const uint32_t key = u[i];
        le += key <= v1 ? 1u : 0u;
        if (key > v1) above = min(above, key);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        le += __shfl_xor(le, o);
        above = min(above, uint32_t(__shfl_xor(above, o)));
    }
    if (lane == 0) {
        sc.hist[wave] = le;
        sc.hist[8 + wave] = above;
    }
    __syncthreads();
    uint32_t tle = 0, tab = 0xffffffffu;
    for (int w = 0; w < kMedThreads / 64; ++w) {
        tle += sc.hist[w];
        tab = min(tab, sc.hist[8 + w]);
    }
    const uint32_t v2 = tle >= r1 + 2 ? v1 : tab;
    return 0.5 * (double(__uint_as_float(v1)) + double(__uint_as_float(v2)));
}

constexpr int kMaxW = 8192;

// One workgroup per block of W bins: X[k] from Z[k] and Z[M - k], then the
// block's median power.
__global__ __launch_bounds__(kMedThreads) void k_unpack_median(const float2 *__restrict__ Z,
                                                               int64_t M, float2 *__restrict__ X,
                                                               double *__restrict__ med, int W) {
    extern __shared__ uint32_t s[];  // W keys (dynamic: the block's size only)
    __shared__ SelectScratch sc;
    const int t = threadIdx.x;
    const int64_t b0 = int64_t(blockIdx.x) * W;
    const int w = int(min(int64_t(W), M - b0));
    const double inv_n = 1.0 / double(2 * M);
    for (int i = t; i < w; i += kMedThreads) {
        const int64_t k = b0 + i;
        float2 x = make_float2(0.f, 0.f);
        if (k > 0) {
            const float2 zk = Z[k];
            const float2 zm = Z[M - k];
            // E = (Z[k] + conj Z[M-k]) / 2,  O = (Z[k] - conj Z[M-k]) / (2i)
            const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            double sn, cs;
            sincospi(-2.0 * double(k) * inv_n, &sn, &cs);
            x = cadd(e, cmul(o, make_float2(float(cs), float(sn))));
        }
        X[k] = x;
        s[i] = __float_as_uint(cnorm(x));
    }
    __syncthreads();
    const double m = median_select(s, w, sc);
    if (t == 0) med[blockIdx.x] = m;
}

__global__ __launch_bounds__(kMedThreads) void k_median(const float2 *__restrict__ X, int64_t nb,
                                                        double *__restrict__ med, int W) {
    extern __shared__ uint32_t s[];  // W keys
    __shared__ SelectScratch sc;
    const int t = threadIdx.x;
    const int64_t b0 = int64_t(blockIdx.x) * W;
    const int w = int(min(int64_t(W), nb - b0));
    for (int i = t; i < w; i += kMedThreads) s[i] = __float_as_uint(cnorm(X[b0 + i]));
    __syncthreads();
    const double m = median_select(s, w, sc);
    if (t == 0) med[blockIdx.x] = m;
}

// -------------------------------------------------------- segment DFTs
// Segment s (one workgroup of fft_threads(LOG2S) threads, lds holding
// FftShape::LDS_FLOAT2 float2): DFT of Xhat[s L - h + n], n in [0, S).
template <int LOG2S, bool SPLIT = false>
__device__ __forceinline__ void segfft_item(float2 *lds, int t, const float2 *__restrict__ X,
                                            const double *__restrict__ med, int W, int64_t nb, int h, int64_t s,
                                            float2 *__restrict__ segspec) {
    using Sh = FftShape<LOG2S, fft_threads(LOG2S)>;
    const int64_t L = seg_valid(Sh::S, h);
    const int64_t g0 = s * L - h;
    const int64_t nblk = (nb + W - 1) / W;
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) {
        const int64_t g = g0 + t + Sh::NT * m;
        float2 x = make_float2(0.f, 0.f);
        if (g >= 0 && g < nb) {
            x = X[g];
            if (med) {
                const double mk = median_curve(med, nblk, W, nb, g);
                const float sc = mk > 0.0 ? float(sqrt(kLn2 / mk)) : 0.f;
                x = make_float2(x.x * sc, x.y * sc);
            }
        }
        v[m] = x;
    }
    fft_wg<Sh, -1, SPLIT>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) segspec[s * Sh::S + t + Sh::NT * m] = v[m];
}

template <int LOG2S>
__global__ __launch_bounds__(fft_threads(LOG2S)) void k_segfft(const float2 *__restrict__ X,
                                                               const double *__restrict__ med,
                                                               int W, int64_t nb, int h,
                                                               float2 *__restrict__ segspec) {
    using Sh = FftShape<LOG2S, fft_threads(LOG2S)>;
    // From 8192 points the one-round exchange (S float2 of LDS) would hold a
    // compute unit to two workgroups, fewer than its registers allow, and
    // the 527 segments of a 2^23-sample series would take two rounds of
    // workgroups: exchange the halves through S floats instead.
    constexpr bool kSplit = LOG2S >= 13;
    __shared__ float2 lds[kSplit ? (Sh::LDS_FLOAT2 + 1) / 2 : Sh::LDS_FLOAT2];
    segfft_item<LOG2S, kSplit>(lds, threadIdx.x, X, med, W, nb, h, blockIdx.x, segspec);
}

// Xhat = X sqrt(ln2 / m(k)) written out (inspection only; the search path
// applies the same scale inside k_segfft's loader).
__global__ __launch_bounds__(256) void k_normalise(const float2 *__restrict__ X, const double *__restrict__ med,
                                                   int W, int64_t nb, float2 *__restrict__ out) {
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (g >= nb) return;
    const int64_t nblk = (nb + W - 1) / W;
    const double mk = median_curve(med, nblk, W, nb, g);
    const float sc = mk > 0.0 ? float(sqrt(kLn2 / mk)) : 0.f;
    const float2 x = X[g];
    out[g] = make_float2(x.x * sc, x.y * sc);
}

// ----------------------------------------------- fused correlation kernel
// Work item u enumerates (group of grp template blocks, segment s, block in
// the group), group-major.  Workgroup i runs item u = (i mod 8) * per + i div 8,
// so each XCD walks a contiguous range of items: when the template blocks split
// evenly over the 8 XCDs, one group of blocks over all segments, with the
// group's templates kept in its own L2 and each segment spectrum read by the
// group's blocks while still resident.
//
// INTERBIN: every template is run twice, with the integer-offset bank and
// with the half-bin bank, into a row of 2 nb floats (bins k in [0, nb), the
// points k + 1/2 in [nb, 2 nb)) and one code per pair (k, k + 1/2).  The first
// pass stores the codes of its own 4 points (one byte each); the second pass
// (same thread, same chunk) reads that word back and keeps the larger code
// of each pair.
// Work item (segment s, template block tb): templates [tb tpb, min(nz, (tb + 1) tpb)).
template <int LOG2S, bool INTERBIN, bool HOLD = false>
__device__ __forceinline__ void correlate_item(float2 *lds, const Twiddles<FftShape<LOG2S, corr_threads(LOG2S)>, +1> &tw,
                                               int t, const float2 *__restrict__ segspec,
                                               const float2 *__restrict__ bank, const float2 *__restrict__ bank_half,
                                               int nz, int tpb, int64_t nb, int h, int64_t s, int64_t tb,
                                               float *__restrict__ plane, uint8_t *__restrict__ codes,
                                               float code_inv) {
    using Sh = FftShape<LOG2S, corr_threads(LOG2S)>;
    const int64_t L = seg_valid(Sh::S, h);
    const int iz0 = int(tb) * tpb;
    const int iz1 = min(nz, iz0 + tpb);
    // HOLD: the segment spectrum is loaded once into registers and reused by
    // every template (at 8192 points 12 % less time than re-reading it per
    // template).  Otherwise it is re-read per template, from L2 (consecutive
    // workgroups of an XCD share it).
    // Operands come through buffer loads: one 32-bit lane offset and a
    // per-point constant offset, no 64-bit address arithmetic per load.
    const __amdgpu_buffer_rsrc_t rsp = buffer_rsrc(segspec + s * Sh::S, Sh::S * 8);

    const int64_t kbase = s * L - h;  // plane column of segment point n is kbase + n
    // points [h, nend) of this segment are plane columns [s L, min(s L + L, nb))
    const int nend = int(min(int64_t(h) + L, nb - kbase));
    const int sh = int(((kbase % 4) + 4) % 4);  // plane row offset of point 0 modulo 4
    constexpr int PASSES = INTERBIN ? 2 : 1;
    float2 xh[HOLD ? Sh::R : 1];
    if constexpr (HOLD) {
#pragma unroll
        for (int m = 0; m < Sh::R; ++m) xh[m] = buffer_load_f2(rsp, t, Sh::NT * m);
    }
    for (int it = iz0 * PASSES; it < iz1 * PASSES; ++it) {
        const int iz = INTERBIN ? (it >> 1) : it;
        const bool second = INTERBIN && (it & 1);
        // Keep the lane offset inside the loop: hoisting the per-point
        // addresses out of it would cost more registers than recomputing.
        int to = t;
        asm volatile("" : "+v"(to));
        const __amdgpu_buffer_rsrc_t rbz = buffer_rsrc((second ? bank_half : bank) + int64_t(iz) * Sh::S, Sh::S * 8);
        // The operand loads go out in two batches of R / 2 points, each
        // batch issued before any of its products is formed (the scheduling
        // barriers keep the compiler from interleaving loads and multiplies,
        // which under register pressure it does by waiting for each pair in
        // turn: one memory round trip per point).
        float2 v[Sh::R];
        static_for<0, 2>([&](auto hc) {
            constexpr int m0 = decltype(hc)::value * (Sh::R / 2);
            float2 b[Sh::R / 2];
#pragma unroll
            for (int m = 0; m < Sh::R / 2; ++m) {
                if constexpr (HOLD) v[m0 + m] = xh[m0 + m];
                else v[m0 + m] = buffer_load_f2(rsp, to, Sh::NT * (m0 + m));
                b[m] = buffer_load_f2(rbz, to, Sh::NT * (m0 + m));
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < Sh::R / 2; ++m) v[m0 + m] = cmul(v[m0 + m], b[m]);
            __builtin_amdgcn_sched_barrier(0);
        });
        fft_wg<Sh, +1>(v, lds, tw, t);
        // Powers through LDS so that each thread stores 4 consecutive
        // points: point n sits at LDS index n + sh, which puts chunk c
        // (indices 4c .. 4c+3) on a 16-byte boundary of the plane row, i.e.
        // on two 2-bin blocks of the codes (L and s L are multiples of 4, so
        // kept chunks are whole).
        float *__restrict__ lf = reinterpret_cast<float *>(lds);
#pragma unroll
        for (int m = 0; m < Sh::R; ++m) lf[sh + to + Sh::NT * m] = cnorm(v[m]);
        __syncthreads();
        constexpr int NCH = (Sh::S + 6) / 4;  // chunks covering indices [0, S + 3)
        if constexpr (!INTERBIN) {
            // Chunk c holds plane columns kbase - sh + 4c .. + 3 and the codes
            // of blocks (kbase - sh) / 2 + 2c, + 1 (kbase - sh is a multiple
            // of 4).  Per-row buffer resources bound the stores to the kept
            // points; three chunks per step so that their LDS reads overlap.
            float *__restrict__ row = plane + int64_t(iz) * nb + kbase;
            uint8_t *__restrict__ qrow = codes + int64_t(iz) * (nb / 2) + (kbase - sh) / 2;
            const __amdgpu_buffer_rsrc_t rrow = buffer_rsrc(row, nend * 4);
            const __amdgpu_buffer_rsrc_t rq = buffer_rsrc(qrow, (nend + sh) / 2);
            constexpr int UNR = 3;
            for (int c0 = t; c0 < NCH; c0 += UNR * Sh::NT) {
                float4 p4[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k)
                    p4[k] = *reinterpret_cast<const float4 *>(lf + 4 * min(c0 + k * Sh::NT, NCH - 1));
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    const int c = c0 + k * Sh::NT;
                    const int n0 = 4 * c - sh;
                    if (c < NCH && n0 >= h && n0 + 4 <= nend) {
                        buffer_store_nt_f4(p4[k], rrow, 4 * n0);
                        buffer_store_nt_u16(block_codes4(p4[k], code_inv), rq, 2 * c);
                    }
                }
            }
        } else {
            float *__restrict__ row = plane + int64_t(iz) * nb * PASSES + (second ? nb : 0) + kbase;
            uint8_t *__restrict__ qrow = codes + int64_t(iz) * (nb * PASSES / 2);
            for (int c = t; c < NCH; c += Sh::NT) {
                const int n0 = 4 * c - sh;
                const float4 p4 = *reinterpret_cast<const float4 *>(lf + 4 * c);
                if (n0 >= h && n0 + 4 <= nend) {
                    __builtin_nontemporal_store(__builtin_bit_cast(f32x4v, p4), reinterpret_cast<f32x4v *>(row + n0));
                    uint32_t q = uint32_t(power_code(p4.x, code_inv)) | (uint32_t(power_code(p4.y, code_inv)) << 8) |
                                 (uint32_t(power_code(p4.z, code_inv)) << 16) |
                                 (uint32_t(power_code(p4.w, code_inv)) << 24);
                    uint32_t *__restrict__ qw = reinterpret_cast<uint32_t *>(qrow + kbase + n0);
                    if (!second) {
                        *qw = q;  // read back by the half-bin pass
                    } else {
                        const uint32_t a = *qw;
                        uint32_t m = 0;
#pragma unroll
                        for (int b = 0; b < 32; b += 8) m |= max((a >> b) & 0xffu, (q >> b) & 0xffu) << b;
                        __builtin_nontemporal_store(m, qw);
                    }
                }
            }
        }
        __syncthreads();  // the next transform writes lds
    }
}

template <int LOG2S, bool INTERBIN>
__global__ __launch_bounds__(corr_threads(LOG2S), corr_waves(LOG2S, INTERBIN)) void k_correlate(
    const float2 *__restrict__ segspec, const float2 *__restrict__ bank, const float2 *__restrict__ bank_half,
    int nz, int tpb, int64_t nb, int h, int64_t nseg, int64_t total, int64_t per, int grp,
    float *__restrict__ plane, uint8_t *__restrict__ codes, float code_inv) {
    using Sh = FftShape<LOG2S, corr_threads(LOG2S)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    const int64_t u = int64_t(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    if (u >= total) return;
    const int64_t gsz = int64_t(grp) * nseg;
    const int64_t gi = u / gsz;
    const int64_t gr = u - gi * gsz;
    const int64_t s = gr / grp;
    const int64_t tb = gi * grp + (gr - s * grp);
    Twiddles<Sh, +1> tw;
    tw.init(t);
    correlate_item<LOG2S, INTERBIN, corr_hold(LOG2S, INTERBIN)>(lds, tw, t, segspec, bank, bank_half, nz, tpb, nb, h,
                                                                 s, tb, plane, codes, code_inv);
}

// ------------------------------------------------ harmonic sum and peaks
struct Thr {
    float v[5];
};

// Every term of every level is a fraction j/16 of the top harmonic
// (j = 1..16, level l >= 1 adds the odd multiples of 16 / 2^l; the cell
// itself is j = 16):
//   column c_j(k) = floor((j k + 8) / 16),
//   row    r_j(iz) = izc + sgn(d) floor((|d| j + 8) / 16),  d = iz - izc,
// the rounding (half away from zero) of k j/16 and d j/16, i.e. of
// k j'/nh and d j'/nh for the j'-th harmonic of an nh-harmonic sum.
// izc < 0: every harmonic lies in the cell's own row (the time-domain search,
// whose resampling removes the drift of all harmonics), row izc + d.
__device__ __forceinline__ int frac_row(int izc, int d, int j) {
    if (izc < 0) return izc + d;
    const int ad = d < 0 ? -d : d;
    const int off = (ad * j + 8) >> 4;
    return d < 0 ? izc - off : izc + off;
}

// S_1, S_2, ..., S_2^LEVELS from the 16 fraction terms v[j] (v[0] unused),
// always in this one summation order.
template <int LEVELS>
__device__ __forceinline__ void nested_sums(const float (&v)[17], float (&s)[5]) {
    s[0] = v[16];
    if constexpr (LEVELS >= 1) s[1] = s[0] + v[8];
    if constexpr (LEVELS >= 2) s[2] = s[1] + (v[4] + v[12]);
    if constexpr (LEVELS >= 3) s[3] = s[2] + ((v[2] + v[6]) + (v[10] + v[14]));
    if constexpr (LEVELS >= 4) s[4] = s[3] + (((v[1] + v[3]) + (v[5] + v[7])) + ((v[9] + v[11]) + (v[13] + v[15])));
}

template <int LEVELS>
__device__ __forceinline__ constexpr bool frac_used(int j) {
    return (j % (16 >> LEVELS)) == 0;
}

// All levels at one cell, loading its terms directly from the plane.
// split > 0: a half-bin plane, whose column c (half bins) is stored at
// c / 2 for even c and at split + c / 2 for odd c (split = bins per row).
template <int LEVELS>
__device__ __forceinline__ void cell_sums(const float *__restrict__ P, int64_t nb, int64_t split, int izc, int iz,
                                          int k, float (&s)[5]) {
    float v[17];
    v[0] = 0.f;
    const int d = iz - izc;
    static_for<1, 17>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (frac_used<LEVELS>(j)) {
            const int64_t c = (j * k + 8) >> 4;
            const int64_t col = split ? (c >> 1) + (c & 1) * split : c;
            v[j] = P[int64_t(frac_row(izc, d, j)) * nb + col];
        } else {
            v[j] = 0.f;
        }
    });
    nested_sums<LEVELS>(v, s);
}

// Pass 1, the screen, on the codes of 2-bin blocks (see block_code): a code
// is at least P / delta for both bins of its block, so for the block of bins
// 2b, 2b + 1 of row iz, sum_j max(codes of the blocks holding c_j(2b) and
// c_j(2b + 1) in row r_j) is at least each bin's power sum / delta.  A block
// whose bounds stay below T_l = floor(thr_l / delta (1 - 1e-5)) at every level
// holds no bin that can reach a threshold.  The others ("flagged") are listed
// twice: as block entries (column pair, row), whose bins 2e and 2e + 1 are the
// cell indices of entry e, and per group of 32 columns of one row (a record
// with the row, the group, a 16-bit mask of its flagged blocks and its first
// cell index; group_map[iz][m] holds the record index of group (m, iz)) for
// the neighbour lookups.  Map entries are written only for flagged groups and
// are trusted only when the record they point to names the same group, so the
// map needs no clearing between searches.
//
// A lane owns the 16 blocks 16 m + beta (32 columns) of a row.  Fraction j of
// bin 2 (16 m + beta) + i lies in block j m + floor((2 j beta + j i + 8) / 32):
// the 16 blocks' codes of fraction j sit in bytes [j m, j m + span) of row r_j
// at compile-time offsets.  Blocks 2p and 2p+1 share one 32-bit register
// (p < 8), one per 16-bit half: a sum of at most 16 codes (<= 4080) never
// carries into the upper half, and a half reaches level l iff
// sum + 0x8000 - T_l sets its bit 15.  All loads of a row are independent of
// each other and issued together.
constexpr int SC_TZ = 8;      // rows per wave
constexpr int SC_WAVES = 4;   // waves per workgroup
constexpr int SC_COLS = 32;   // columns per lane (one group)
constexpr int SC_WAVE_COLS = 64 * SC_COLS;

struct ScreenThr {
    uint32_t k[5];  // (0x8000 - T_l) in both 16-bit halves
};

struct Group {
    int32_t m;         // columns 32 m .. 32 m + 31
    uint32_t iz_mask;  // row in bits 0..15, flagged 2-column blocks in bits 16..31
    uint32_t first;    // cell index of the group's first flagged bin
    uint32_t pad;
};

// Counters (six 32-bit words, zeroed before the pass): candidates; (unused);
// overflow flag; (unused); flagged cells (low word) and groups (high word) of
// one 64-bit counter, so that a wave reserves both with one atomic.
enum { CNT_CANDS = 0, CNT_OVERFLOW = 2, CNT_PAIR = 4 };

__device__ __forceinline__ uint32_t cell_count(const uint32_t *cnt) { return cnt[CNT_PAIR]; }
__device__ __forceinline__ uint32_t group_count(const uint32_t *cnt) { return cnt[CNT_PAIR + 1]; }

// Byte layout of one fraction's 16 block codes.
template <int J>
struct FracBlocks {
    static constexpr int lo(int b) { return (2 * J * b + 8) >> 5; }      // block of bin 2 b
    static constexpr int hi(int b) { return (2 * J * b + J + 8) >> 5; }  // block of bin 2 b + 1
    static constexpr int span = hi(15) + 1;                              // bytes used
    static constexpr int maxshift = J % 4 == 0 ? 0 : J % 2 == 0 ? 2 : 3;  // (j m) mod 4
    static constexpr int nd = (maxshift + span + 3) / 4;                 // dwords loaded
    static constexpr int nw = (span + 3) / 4;                            // aligned words
};

// Level group of fraction j: the level that first adds it (16 -> 0, 8 -> 1,
// 4 and 12 -> 2, 2 mod 4 -> 3, odd -> 4).
constexpr int frac_level(int j) { return j == 16 ? 0 : j % 2 ? 4 : j % 4 ? 3 : j % 8 ? 2 : 1; }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per-half maximum of two pairs of 16-bit values.
__device__ __forceinline__ uint32_t max_u16x2(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_max(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}

// Bytes A and C of the aligned words w (C >> 2 is A >> 2 or one more) in the
// low bytes of the two 16-bit halves of the result.
template <int A, int C, int NW>
__device__ __forceinline__ uint32_t gather2(const uint32_t (&w)[NW]) {
    constexpr int wa = A >> 2, wc = C >> 2;
    static_assert(wc == wa || wc == wa + 1, "bytes in adjacent words");
    // v_perm_b32 selector bytes: 0-3 pick bytes of the second source, 4-7
    // bytes of the first, 0x0c gives zero.
    constexpr uint32_t sel = uint32_t(A & 3) | 0x0c00u | (uint32_t((wc == wa ? 0 : 4) + (C & 3)) << 16) | 0x0c000000u;
    return __builtin_amdgcn_perm(w[wc], w[wa], sel);
}

// Add fraction J's bounds of the lane's 8 block pairs (group m of row qrow) to acc.
template <int J>
__device__ __forceinline__ void add_fraction(const uint8_t *__restrict__ qrow, int64_t m, uint32_t (&acc)[8]) {
    using FB = FracBlocks<J>;
    const int64_t b = int64_t(J) * m;  // first byte
    const uint32_t *__restrict__ src = reinterpret_cast<const uint32_t *>(qrow + (b & ~int64_t(3)));
    uint32_t d[FB::nd];
#pragma unroll
    for (int q = 0; q < FB::nd; ++q) d[q] = src[q];
    uint32_t w[FB::nw];
    if constexpr (FB::maxshift == 0) {
#pragma unroll
        for (int q = 0; q < FB::nw; ++q) w[q] = d[q];
    } else {
        const uint32_t sh = uint32_t(b & 3);
#pragma unroll
        for (int q = 0; q < FB::nw; ++q) w[q] = __builtin_amdgcn_alignbyte(d[q + 1 < FB::nd ? q + 1 : q], d[q], sh);
    }
    static_for<0, 8>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int l0 = FB::lo(2 * p), l1 = FB::lo(2 * p + 1), h0 = FB::hi(2 * p), h1 = FB::hi(2 * p + 1);
        uint32_t v = gather2<l0, l1>(w);
        if constexpr (h0 != l0 || h1 != l1) v = max_u16x2(v, gather2<h0, h1>(w));
        acc[p] += v;
    });
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ uint32_t wave_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Screen tile (bx, by) of a workgroup of 64 SC_WAVES threads: columns
// [bx SC_WAVES 2048, + SC_WAVES 2048), rows [by SC_TZ, + SC_TZ).  rowmask_lds:
// SC_WAVES SC_TZ 64 words of LDS.
template <int LEVELS>
__device__ __forceinline__ void screen_tile(uint32_t *rowmask_lds, int64_t bx, int by, const uint8_t *__restrict__ Q,
                                            int nz, int64_t nb, int izc, const ScreenThr &T,
                                            Group *__restrict__ groups, uint2 *__restrict__ blocks,
                                            uint32_t *__restrict__ group_map, uint32_t *__restrict__ cnt,
                                            uint32_t group_cap, uint32_t cell_cap) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // a workgroup covers SC_WAVES * 2048 columns and SC_TZ rows
    const int64_t m = (bx * SC_WAVES + wave) * 64 + lane;  // column group
    const int iz0 = by * SC_TZ;
    const int64_t ngr = nb / SC_COLS;
    const int64_t qlen = nb / 2;  // codes per row
    const bool valid = m < ngr;
    if (!__any(valid) || iz0 >= nz) return;
    const int64_t mm = valid ? m : 0;  // lanes past the end read group 0 and report nothing
    uint32_t *__restrict__ rowmask = rowmask_lds + wave * (SC_TZ * 64) + lane;  // row r at rowmask[64 r]
    uint32_t mycells = 0, mygroups = 0;
#pragma unroll 1
    for (int r = 0; r < SC_TZ; ++r) {
        const int iz = iz0 + r;
        rowmask[64 * r] = 0;
        if (iz >= nz) continue;
        const int d = iz - izc;
        uint32_t G[LEVELS + 1][8];
#pragma unroll
        for (int l = 0; l <= LEVELS; ++l)
#pragma unroll
            for (int p = 0; p < 8; ++p) G[l][p] = 0u;
        static_for<1, 17>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (frac_used<LEVELS>(j))
                add_fraction<j>(Q + int64_t(frac_row(izc, d, j)) * qlen, mm, G[frac_level(j)]);
        });
        uint32_t mask = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            uint32_t sm = G[0][p];
            uint32_t fl = sm + T.k[0];
#pragma unroll
            for (int l = 1; l <= LEVELS; ++l) {
                sm += G[l][p];
                fl |= sm + T.k[l];
            }
            mask |= ((fl >> 15) & 1u) << (2 * p);
            mask |= (fl >> 31) << (2 * p + 1);
        }
        if (!valid) mask = 0;
        rowmask[64 * r] = mask;
        mycells += 2u * __popc(mask);
        mygroups += mask != 0 ? 1u : 0u;
    }
    // One group record per (lane, row) with flagged blocks; a lane's records
    // and cells get consecutive indices.  One atomic per wave reserves both
    // lists; crossing a capacity raises the overflow flag at once (so a count
    // that later wraps cannot hide it).  (Each lane reads back only its own
    // LDS words, so no barrier is needed.)
    if (!__any(mycells != 0)) return;
    // cells (<= 32 SC_TZ 64 = 16384) in the low half, groups in the high half
    const uint32_t incl = wave_scan((mygroups << 16) | mycells, lane);
    const uint32_t total = __shfl(incl, 63);
    uint32_t cbase = 0, gbase = 0;
    if (lane == 0) {
        const uint32_t tc = total & 0xffffu, tg = total >> 16;
        const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long *>(cnt + CNT_PAIR),
                                                 (static_cast<unsigned long long>(tg) << 32) | tc);
        cbase = uint32_t(old);
        gbase = uint32_t(old >> 32);
        if (uint64_t(cbase) + tc > cell_cap || uint64_t(gbase) + tg > group_cap) cnt[CNT_OVERFLOW] = 1u;
    }
    uint32_t first = __shfl(cbase, 0) + (incl & 0xffffu) - mycells;
    uint32_t g = __shfl(gbase, 0) + (incl >> 16) - mygroups;
#pragma unroll 1
    for (int r = 0; r < SC_TZ; ++r) {
        const uint32_t mask = rowmask[64 * r];
        if (mask == 0) continue;
        const uint32_t ncell = 2u * __popc(mask);
        const int iz = iz0 + r;
        const bool fits = uint64_t(first) + ncell <= cell_cap;
        // every record below min(count, group_cap) is written, with no cells
        // when they do not fit (the overflow flag reports the loss)
        if (g < group_cap) {
            groups[g] = Group{int32_t(m), uint32_t(iz) | ((fits ? mask : 0u) << 16), first, 0u};
            if (fits) group_map[int64_t(iz) * ngr + m] = g;
        }
        if (fits) {
            uint32_t e = first >> 1;
            for (uint32_t bm = mask; bm; bm &= bm - 1u, ++e)
                blocks[e] = make_uint2(uint32_t(m * (SC_COLS / 2) + __ffs(bm) - 1), uint32_t(iz));
        }
        ++g;
        first += ncell;
    }
}

template <int LEVELS>
__global__ __launch_bounds__(64 * SC_WAVES) void k_screen(const uint8_t *__restrict__ Q, int nz, int64_t nb,
                                                          int izc, ScreenThr T, Group *__restrict__ groups,
                                                          uint2 *__restrict__ blocks, uint32_t *__restrict__ group_map,
                                                          uint32_t *__restrict__ cnt, uint32_t group_cap,
                                                          uint32_t cell_cap) {
    // Row masks of the waves, kept until their records are written.
    __shared__ uint32_t rowmask_lds[SC_WAVES * SC_TZ * 64];
    screen_tile<LEVELS>(rowmask_lds, blockIdx.x, blockIdx.y, Q, nz, nb, izc, T, groups, blocks, group_map, cnt,
                        group_cap, cell_cap);
}

constexpr int SUM_STRIDE = 5;  // floats per flagged cell in the sums array

// Cell index of bin i (< 32) of a group, when its block is flagged.
__device__ __forceinline__ bool cell_flagged(const Group &r, int i) { return (r.iz_mask >> (16 + (i >> 1))) & 1u; }
__device__ __forceinline__ uint32_t cell_index(const Group &r, int i) {
    const uint32_t bm = r.iz_mask >> 16;
    return r.first + 2u * uint32_t(__popc(bm & ((1u << (i >> 1)) - 1u))) + uint32_t(i & 1);
}

// Pass 2, one lane per flagged cell: its exact FP32 sums, loaded from the
// plane in the one summation order of nested_sums.  No list is built: the
// neighbour test reads every flagged cell's sums and keeps the ones that
// reach a threshold (a hit list reserved with one atomic per workgroup step
// cost 70 us on a trial with strong pulsars: every step of every workgroup
// contended on the one counter).
// Exact-sum workgroup wg of nwg (256 threads): flagged cells wg 256 + i,
// stepping by nwg 256.
template <int LEVELS>
__device__ __forceinline__ void exact_tile(uint32_t wg, uint32_t nwg, const float *__restrict__ P, int nz, int64_t nb,
                                           int64_t split, int izc, const uint2 *__restrict__ blocks,
                                           const uint32_t *__restrict__ cnt, uint32_t cell_cap,
                                           float *__restrict__ sums) {
    const uint32_t nc = min(cell_count(cnt), cell_cap);
    for (uint32_t c = wg * 256u + threadIdx.x; c < nc; c += nwg * 256u) {
        const uint2 e = blocks[c >> 1];
        const int64_t k = 2 * int64_t(e.x) + (c & 1);
        const int iz = int(e.y);
        if (k < nb && iz < nz) {  // guards against entries of an overflowed list
            float sv[5];
            cell_sums<LEVELS>(P, nb, split, izc, iz, int(k), sv);
            float *__restrict__ o = sums + int64_t(c) * SUM_STRIDE;
#pragma unroll
            for (int l = 0; l <= LEVELS; ++l) o[l] = sv[l];
        }
    }
}

template <int LEVELS>
__global__ __launch_bounds__(256) void k_exact(const float *__restrict__ P, int nz, int64_t nb, int64_t split,
                                               int izc, const uint2 *__restrict__ blocks,
                                               const uint32_t *__restrict__ cnt, uint32_t cell_cap,
                                               float *__restrict__ sums) {
    exact_tile<LEVELS>(blockIdx.x, gridDim.x, P, nz, nb, split, izc, blocks, cnt, cell_cap, sums);
}

// Candidate records staged in LDS by a neighbour-test workgroup before one
// atomic reserves their slots (8 KB: the workgroups of a CU stay limited by
// their waves, not by LDS).
constexpr uint32_t PK_STAGE = 512;

// Pass 3, one lane per hit: the 3x3 local maximum at every level the cell
// reaches.  A cell keeps a level when it is strictly greater than the
// neighbours earlier in row-major (iz, k) order and at least equal to the
// later ones; neighbours outside the plane are ignored.  A neighbour that was
// not flagged has sums below every threshold, hence below the cell's, and is
// beaten without being looked at; the others are found through the group map
// (map entry, record, sums, issued side by side for the 8 neighbours).
// Neighbour-test workgroup wg of nwg (256 threads): flagged cells wg 256 + i,
// stepping by nwg 256; stage: PK_STAGE records of LDS.  A workgroup stages
// its candidates and reserves their slots with one atomic when the stage
// would overflow and once at the end.
template <int LEVELS>
__device__ __forceinline__ void peaks_tile(uint32_t wg, uint32_t nwg, int nz, int64_t nb, Thr thr, const Group *__restrict__ groups,
                                               const uint32_t *__restrict__ group_map, const uint2 *__restrict__ blocks,
                                               const float *__restrict__ sums, uint32_t *__restrict__ cnt,
                                               uint32_t group_cap, uint32_t cell_cap, DevCand *__restrict__ cands,
                                               uint32_t cap, DevCand *stage) {
    __shared__ uint32_t wsum[2][4];  // per-wave candidate counts, by iteration parity
    __shared__ uint32_t gbase;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t nc = min(cell_count(cnt), cell_cap);
    const uint32_t ng = min(group_count(cnt), group_cap);
    const int64_t ngr = nb / SC_COLS;
    // staged records (the same value in every thread)
    uint32_t staged = 0;
    auto flush = [&]() {
        if (threadIdx.x == 0) gbase = atomicAdd(cnt + CNT_CANDS, staged);
        __syncthreads();
        const uint32_t g = gbase;
        for (uint32_t i = threadIdx.x; i < staged; i += 256u)
            if (g + i < cap) cands[g + i] = stage[i];
        __syncthreads();  // the stage and gbase are rewritten after this
        staged = 0;
    };
    int par = 0;
    // the bounds of this loop are the same for every thread of the workgroup
    for (uint32_t cw = wg * 256u; cw < nc; cw += nwg * 256u, par ^= 1) {
        const uint32_t c = cw + threadIdx.x;
        uint32_t lmask = 0;  // levels still alive
        int64_t k = 0;
        int iz = 0;
        float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if (c < nc) {
            const uint2 e = blocks[c >> 1];
            k = 2 * int64_t(e.x) + (c & 1);
            iz = int(e.y);
            if (k < nb && iz < nz) {  // the exact pass wrote no sums for other entries
                const float *__restrict__ o = sums + int64_t(c) * SUM_STRIDE;
#pragma unroll
                for (int l = 0; l <= LEVELS; ++l) {
                    s[l] = o[l];
                    if (s[l] >= thr.v[l]) lmask |= 1u << l;
                }
            }
        }
        if (lmask != 0) {
            // neighbour n = 3 (di + 1) + (dk + 1), n != 4
            uint32_t gi[9];
#pragma unroll
            for (int n = 0; n < 9; ++n) {
                const int di = n / 3 - 1, dk = n % 3 - 1;
                gi[n] = ~0u;
                if (n == 4) continue;
                const int iz2 = iz + di;
                const int64_t k2 = k + dk;
                if (iz2 < 0 || iz2 >= nz || k2 < 0 || k2 >= nb) continue;
                gi[n] = group_map[int64_t(iz2) * ngr + k2 / SC_COLS];
            }
            Group rn[9];
#pragma unroll
            for (int n = 0; n < 9; ++n) {
                rn[n] = Group{-1, 0u, 0u, 0u};
                if (gi[n] < ng) rn[n] = groups[gi[n]];
            }
            float sn[9][5];
            bool use[9];
#pragma unroll
            for (int n = 0; n < 9; ++n) {
                const int di = n / 3 - 1, dk = n % 3 - 1;
                const int64_t k2 = k + dk;
                const int i2 = int(k2 % SC_COLS);
                use[n] = gi[n] < ng && int64_t(rn[n].m) == k2 / SC_COLS &&
                         (rn[n].iz_mask & 0xffffu) == uint32_t(iz + di) && cell_flagged(rn[n], i2) &&
                         uint64_t(rn[n].first) + 2u * uint32_t(__popc(rn[n].iz_mask >> 16)) <= cell_cap;
#pragma unroll
                for (int l = 0; l <= LEVELS; ++l) sn[n][l] = 0.f;
                if (use[n]) {
                    const float *__restrict__ o2 = sums + int64_t(cell_index(rn[n], i2)) * SUM_STRIDE;
#pragma unroll
                    for (int l = 0; l <= LEVELS; ++l) sn[n][l] = o2[l];
                }
            }
#pragma unroll
            for (int n = 0; n < 9; ++n) {
                if (!use[n]) continue;
                const bool earlier = n < 4;
#pragma unroll
                for (int l = 0; l <= LEVELS; ++l) {
                    const bool beaten = earlier ? !(s[l] > sn[n][l]) : !(s[l] >= sn[n][l]);
                    if (beaten) lmask &= ~(1u << l);
                }
            }
        }
        const uint32_t ncand = __popc(lmask);
        const uint32_t incl = wave_scan(ncand, lane);
        if (lane == 63) wsum[par][wave] = incl;
        // orders the counts, and the previous step's staged records before a flush
        __syncthreads();
        const uint32_t tot = wsum[par][0] + wsum[par][1] + wsum[par][2] + wsum[par][3];
        if (staged + tot > PK_STAGE) flush();
        uint32_t slot = incl - ncand;
        for (int w = 0; w < wave; ++w) slot += wsum[par][w];
        if (tot > PK_STAGE) {
            // a step with more records than the stage holds (up to 256 x 5)
            // reserves and writes them directly
            if (threadIdx.x == 0) gbase = atomicAdd(cnt + CNT_CANDS, tot);
            __syncthreads();
            slot += gbase;
#pragma unroll
            for (int l = 0; l <= LEVELS; ++l) {
                if ((lmask >> l) & 1u) {
                    if (slot < cap) cands[slot] = DevCand{int32_t(k), iz, 1 << l, s[l]};
                    ++slot;
                }
            }
            __syncthreads();  // gbase is rewritten after this
        } else {
            slot += staged;
#pragma unroll
            for (int l = 0; l <= LEVELS; ++l) {
                if ((lmask >> l) & 1u) stage[slot++] = DevCand{int32_t(k), iz, 1 << l, s[l]};
            }
            staged += tot;
        }
    }
    if (staged) {
        __syncthreads();  // the last step's records are staged
        flush();
    }
}

template <int LEVELS>
__global__ __launch_bounds__(256) void k_peaks(int nz, int64_t nb, Thr thr, const Group *__restrict__ groups,
                                               const uint32_t *__restrict__ group_map, const uint2 *__restrict__ blocks,
                                               const float *__restrict__ sums, uint32_t *__restrict__ cnt,
                                               uint32_t group_cap, uint32_t cell_cap, DevCand *__restrict__ cands,
                                               uint32_t cap) {
    __shared__ DevCand stage[PK_STAGE];
    peaks_tile<LEVELS>(blockIdx.x, gridDim.x, nz, nb, thr, groups, group_map, blocks, sums, cnt, group_cap, cell_cap,
                       cands, cap, stage);
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}


// ------------------------------------------------- persistent batch kernel
// Scratch layout of the harmonic-sum passes (launch_harmsum's order).
struct HarmLists {
    Group *groups;
    float *sums;
    uint2 *blocks;
    uint32_t *group_map;
};
__device__ __forceinline__ HarmLists harm_lists(void *scratch, uint32_t cell_cap, uint32_t group_cap) {
    HarmLists r;
    r.groups = static_cast<Group *>(scratch);
    r.sums = reinterpret_cast<float *>(r.groups + group_cap);
    r.blocks = reinterpret_cast<uint2 *>(r.sums + size_t(cell_cap) * SUM_STRIDE);
    r.group_map = reinterpret_cast<uint32_t *>(r.blocks + cell_cap / 2);
    return r;
}

struct BatchArgs {
    const BatchTrial *trials;
    const uint32_t *tiles;
    uint32_t *ctl;
    const float2 *bank;
    int ntrials, slots, nz, tpb, h, W, izc;
    uint32_t ntiles, cell_cap, group_cap, cand_cap;
    float code_inv;
    Thr thr;
    ScreenThr T;
};

// A dependency wait gives up after this long (device wall clock, 100 MHz
// ticks: 1 s), orders of magnitude above the longest legitimate wait (one
// trial's correlation), and raises the error flag.  Bounded in time, not in
// polls: under contention one poll can take long.
constexpr uint64_t kBatchWaitTicks = 100000000ull;

// Counter value as the device's coherence point holds it: an atomic add of
// zero (a read-modify-write is performed where every XCD's atomics are,
// which a plain load need not see at once).
__device__ __forceinline__ uint32_t coherent_read(uint32_t *p) {
    return __hip_atomic_fetch_add(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Executed by all lanes of one wave together (the loop condition is
// wave-uniform).  Waits until *done >= target, then one acquire fence at
// agent scope so that the producers' results are visible to the whole
// workgroup after its next barrier.  False when the error flag is raised, by
// this wait running out (which records what it waited for in ctl[2..5]) or by
// another workgroup's.
__device__ __forceinline__ bool batch_wait(uint32_t *done, uint32_t target, uint32_t *ctl, uint32_t stage,
                                           uint32_t trial) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 0;; ++it) {
        const uint32_t v = __builtin_amdgcn_readfirstlane(coherent_read(done));
        if (v >= target) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return true;
        }
        if ((it & 15u) == 15u) {
            if (__builtin_amdgcn_readfirstlane(coherent_read(ctl + 1)) != 0u) return false;
            if (wall_clock64() - t0 > kBatchWaitTicks) {
                uint32_t first = 1u;
                if (threadIdx.x == 0) first = atomicCAS(ctl + 1, 0u, 1u);
                if (__builtin_amdgcn_readfirstlane(first) == 0u && threadIdx.x == 0) {
                    ctl[2] = stage;
                    ctl[3] = trial;
                    ctl[4] = v;
                    ctl[5] = target;
                }
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(32);
    }
}

// The trial descriptor in scalar registers.  Its fields come from memory
// that the kernel also writes, so the compiler cannot prove them uniform: it
// would keep them in vector registers and turn every buffer access through a
// resource built from them into a loop over the lanes' distinct values.
__device__ __forceinline__ BatchTrial uniform_trial(const BatchTrial *p) {
    constexpr int NW = sizeof(BatchTrial) / 4;
    static_assert(sizeof(BatchTrial) % 4 == 0, "whole words");
    uint32_t w[NW];
    __builtin_memcpy(w, p, sizeof(BatchTrial));
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    BatchTrial r;
    __builtin_memcpy(&r, w, sizeof(BatchTrial));
    return r;
}

// Workgroups take tiles of the global order from ctl[0]; see
// launch_batch_persistent.  Correlation tiles of a trial walk its segments
// template block by template block, so that every XCD keeps one block's
// templates in its L2 while the segment spectra stream past.
template <int LOG2S, int LEVELS>
__global__ __launch_bounds__(256, 2) void k_batch(BatchArgs a) {
    using Sh = FftShape<LOG2S, 256>;
    static_assert(corr_threads(LOG2S) == 256 && fft_threads(LOG2S) == 256, "256-thread transforms");
    static_assert(SC_WAVES * 64 == 256, "screen tiles of 256 threads");
    static_assert(Sh::LDS_FLOAT2 * 2 >= SC_WAVES * SC_TZ * 64, "screen masks fit the transform buffer");
    static_assert(Sh::LDS_FLOAT2 * sizeof(float2) >= PK_STAGE * sizeof(DevCand), "candidates fit the transform buffer");
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    __shared__ uint32_t tinfo[3];
    const int t = threadIdx.x;
    uint32_t *const err = a.ctl + 1;
    uint32_t *const done = a.ctl + kBatchCtlHead;
    const int n = a.ntrials;
    // Wave 0 (all its lanes, under a wave-uniform branch) completes the
    // previous tile and takes the next one; no lane-divergent region holds a
    // barrier or spans the loop's back edge, so every wave runs the same
    // sequence of barriers.
    const uint32_t wave = __builtin_amdgcn_readfirstlane(uint32_t(threadIdx.x) >> 6);
    uint32_t prev_stage = BST_N, prev_trial = 0;
    for (;;) {
        if (wave == 0) {
            if (prev_stage < BST_N) {  // release the previous tile
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                // the L2 write-back has completed before the count moves
                // (the fence's own wait can be dropped as redundant when no
                // store is outstanding)
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                if (t == 0)
                    __hip_atomic_fetch_add(done + prev_stage * n + prev_trial, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            uint32_t stage = BST_N, trial = 0, idx = 0;
            if (__builtin_amdgcn_readfirstlane(coherent_read(err)) == 0u) {
                uint32_t tile = 0;
                if (t == 0) tile = atomicAdd(a.ctl, 1u);
                tile = __builtin_amdgcn_readfirstlane(tile);
                if (tile < a.ntiles) {
                    const uint32_t w = __builtin_amdgcn_readfirstlane(a.tiles[tile]);
                    stage = w >> 29;
                    trial = (w >> 23) & 63u;
                    idx = w & (kBatchMaxStageTiles - 1u);
                    const BatchTrial *tr = a.trials;
                    bool ok = stage < BST_N && int(trial) < n && idx < tr[trial].ntile[stage];
                    if (!ok) {
                        if (t == 0) atomicCAS(err, 0u, 2u);  // malformed order
                    } else if (stage == BST_CORR) {
                        ok = batch_wait(done + BST_SEG * n + trial, tr[trial].ntile[BST_SEG], a.ctl, BST_SEG, trial);
                        if (ok && int(trial) >= a.slots) {
                            const uint32_t prev = trial - uint32_t(a.slots);  // the slot's last user
                            ok = batch_wait(done + BST_PEAK * n + prev, tr[prev].ntile[BST_PEAK], a.ctl, BST_PEAK,
                                            prev);
                        }
                    } else if (stage != BST_SEG) {
                        ok = batch_wait(done + (stage - 1) * n + trial, tr[trial].ntile[stage - 1], a.ctl, stage - 1,
                                        trial);
                    }
                    if (!ok) stage = BST_N;
                }
            }
            if (t == 0) {
                tinfo[0] = stage;
                tinfo[1] = trial;
                tinfo[2] = idx;
            }
        }
        __syncthreads();
        // workgroup-uniform: in scalar registers, so that the trial's
        // descriptor is read with scalar loads
        const uint32_t stage = __builtin_amdgcn_readfirstlane(tinfo[0]);
        const uint32_t trial = __builtin_amdgcn_readfirstlane(tinfo[1]);
        const uint32_t idx = __builtin_amdgcn_readfirstlane(tinfo[2]);
        if (stage >= BST_N) break;
        const BatchTrial tr = uniform_trial(a.trials + trial);
        // The thread index made opaque per tile, so that the twiddles of the
        // transform tiles are computed per tile instead of being hoisted out
        // of the loop (both directions' tables held across every tile would
        // not fit the register file).
        int to = t;
        asm volatile("" : "+v"(to));
        if (stage == BST_SEG) {
            segfft_item<LOG2S>(lds, to, tr.X, tr.med, a.W, tr.nb, a.h, int64_t(idx), tr.seg);
        } else if (stage == BST_CORR) {
            const int64_t s = int64_t(idx) % tr.nseg, tb = int64_t(idx) / tr.nseg;
            Twiddles<Sh, +1> tw;
            tw.init(to);
            // the segment spectrum held in registers (256 VGPRs, no spills:
            // 12 % more trials per second at 8192 points)
            correlate_item<LOG2S, false, true>(lds, tw, to, tr.seg, a.bank, nullptr, a.nz, a.tpb, tr.nb, a.h, s, tb,
                                               tr.plane, tr.codes, a.code_inv);
        } else {
            const HarmLists hl = harm_lists(tr.hits, a.cell_cap, a.group_cap);
            if (stage == BST_SCREEN) {
                const int64_t ncolt = (tr.nb + int64_t(SC_WAVE_COLS) * SC_WAVES - 1) / (int64_t(SC_WAVE_COLS) * SC_WAVES);
                screen_tile<LEVELS>(reinterpret_cast<uint32_t *>(lds), int64_t(idx) % ncolt, int(int64_t(idx) / ncolt),
                                    tr.codes, a.nz, tr.nb, a.izc, a.T, hl.groups, hl.blocks, hl.group_map, tr.cnt,
                                    a.group_cap, a.cell_cap);
            } else if (stage == BST_EXACT) {
                exact_tile<LEVELS>(idx, kBatchExactTiles, tr.plane, a.nz, tr.nb, 0, a.izc, hl.blocks, tr.cnt,
                                   a.cell_cap, hl.sums);
            } else {
                peaks_tile<LEVELS>(idx, kBatchPeakTiles, a.nz, tr.nb, a.thr, hl.groups, hl.group_map, hl.blocks,
                                   hl.sums, tr.cnt, a.group_cap, a.cell_cap, tr.cands, a.cand_cap,
                                   reinterpret_cast<DevCand *>(lds));
            }
        }
        // Every wave's stores have reached the L2 before thread 0 releases
        // the tile at the top of the next iteration (the release writes the
        // L2 back for the other XCDs).
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        prev_stage = stage;
        prev_trial = trial;
    }
}

// ------------------------------------------------------------ dispatch

#define FDAS_SWITCH_LOG2(L, CALL) \
    switch (L) {                  \
        case 6: CALL(6); break;   \
        case 7: CALL(7); break;   \
        case 8: CALL(8); break;   \
        case 9: CALL(9); break;   \
        case 10: CALL(10); break; \
        case 11: CALL(11); break; \
        case 12: CALL(12); break; \
        case 13: CALL(13); break; \
        default: return hipErrorInvalidValue; \
    }

#define FDAS_SWITCH_LOG2_GROUPED(L, CALL) \
    switch (L) {                          \
        case 7: CALL(7); break;           \
        case 8: CALL(8); break;           \
        case 9: CALL(9); break;           \
        case 10: CALL(10); break;         \
        case 11: CALL(11); break;         \
        default: return hipErrorInvalidValue; \
    }

}  // namespace

hipError_t launch_dft(int log2n, int dir, int64_t batch, const float2 *in, float2 *out, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    if (batch > 0x7fffffff) return hipErrorInvalidValue;
#define CALL(L)                                                                                        \
    if (dir < 0)                                                                                       \
        hipLaunchKernelGGL((k_dft<L, -1>), dim3(unsigned(batch)), dim3(fft_threads(L)), 0, st, in, out); \
    else                                                                                               \
        hipLaunchKernelGGL((k_dft<L, +1>), dim3(unsigned(batch)), dim3(fft_threads(L)), 0, st, in, out);
    FDAS_SWITCH_LOG2(log2n, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_r2c_packed(const float *x, int64_t nsamp, float2 *Z, float2 *work, hipStream_t st) {
    const float2 *z = reinterpret_cast<const float2 *>(x);
    int log2m = 0;
    while ((int64_t(1) << log2m) < nsamp / 2) ++log2m;
    if ((int64_t(1) << log2m) != nsamp / 2 || log2m < 6 || log2m > 26) return hipErrorInvalidValue;
    if (log2m <= 13) {
#define CALL(L) hipLaunchKernelGGL((k_r2c_small<L>), dim3(1), dim3(fft_threads(L)), 0, st, z, Z);
        FDAS_SWITCH_LOG2(log2m, CALL)
#undef CALL
        return hipGetLastError();
    }
    const int l1 = (log2m + 1) / 2, l2 = log2m / 2;  // 7 <= l2 <= l1 <= 13
    const unsigned ncols = 1u << l2, nrows = 1u << l1;
    if (l1 <= 11) {  // four columns per workgroup (ncols is a multiple of 4)
#define CALL(L) hipLaunchKernelGGL((k_r2c_cols4<L>), dim3(ncols / kR2cGroup), dim3(fft_threads(L) * kR2cGroup), 0, st, \
                           z, work, l2);
        FDAS_SWITCH_LOG2_GROUPED(l1, CALL)
#undef CALL
    } else {
#define CALL(L) hipLaunchKernelGGL((k_r2c_cols<L>), dim3(ncols), dim3(fft_threads(L)), 0, st, z, work, l2);
        FDAS_SWITCH_LOG2(l1, CALL)
#undef CALL
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (l2 <= 11) {
#define CALL(L) hipLaunchKernelGGL((k_r2c_rows4<L>), dim3(nrows / kR2cGroup), dim3(fft_threads(L) * kR2cGroup), 0, st, \
                           work, Z, l1);
        FDAS_SWITCH_LOG2_GROUPED(l2, CALL)
#undef CALL
    } else {
#define CALL(L) hipLaunchKernelGGL((k_r2c_rows<L>), dim3(nrows), dim3(fft_threads(L)), 0, st, work, Z, l1);
        FDAS_SWITCH_LOG2(l2, CALL)
#undef CALL
    }
    return hipGetLastError();
}

hipError_t launch_unpack_median(const float2 *Z, int64_t nsamp, float2 *X, double *med, int W, hipStream_t st) {
    const int64_t M = nsamp / 2;
    if (W < 2 || W > kMaxW || (W & (W - 1))) return hipErrorInvalidValue;
    const int64_t nblk = (M + W - 1) / W;
    hipLaunchKernelGGL(k_unpack_median, dim3(unsigned(nblk)), dim3(kMedThreads), size_t(W) * sizeof(uint32_t), st, Z,
                       M, X, med, W);
    return hipGetLastError();
}

hipError_t launch_median(const float2 *X, int64_t nb, double *med, int W, hipStream_t st) {
    if (W < 2 || W > kMaxW || (W & (W - 1))) return hipErrorInvalidValue;
    const int64_t nblk = (nb + W - 1) / W;
    hipLaunchKernelGGL(k_median, dim3(unsigned(nblk)), dim3(kMedThreads), size_t(W) * sizeof(uint32_t), st, X, nb,
                       med, W);
    return hipGetLastError();
}

hipError_t launch_segfft(const float2 *X, const double *med, int W, int64_t nb, int log2s, int h,
                         int64_t nseg, float2 *segspec, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
#define CALL(L) \
    hipLaunchKernelGGL((k_segfft<L>), dim3(unsigned(nseg)), dim3(fft_threads(L)), 0, st, X, med, W, nb, h, segspec);
    FDAS_SWITCH_LOG2(log2s, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_normalise(const float2 *X, const double *med, int W, int64_t nb, float2 *out, hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normalise, dim3(unsigned((nb + 255) / 256)), dim3(256), 0, st, X, med, W, nb, out);
    return hipGetLastError();
}

hipError_t launch_correlate(const float2 *segspec, const float2 *bank, const float2 *bank_half, int nz, int tpb,
                            int64_t nb, int log2s, int h, int64_t nseg, float *plane, uint8_t *codes, float code_inv,
                            hipStream_t st) {
    if (nseg <= 0 || nz <= 0) return hipSuccess;
    if (tpb <= 0) return hipErrorInvalidValue;
    const int64_t nzb = (nz + tpb - 1) / tpb;
    const int64_t total = nzb * nseg;
    const int64_t per = (total + kXcds - 1) / kXcds;
    const int64_t grid = per * kXcds;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    // template blocks per group: the blocks of one XCD when they split evenly
    const int grp = (nzb % kXcds == 0) ? int(nzb / kXcds) : 1;
#define CALL(L)                                                                                          \
    if (bank_half)                                                                                       \
        hipLaunchKernelGGL((k_correlate<L, true>), dim3(unsigned(grid)), dim3(corr_threads(L)), 0, st, segspec, \
                           bank, bank_half, nz, tpb, nb, h, nseg, total, per, grp, plane, codes, code_inv);     \
    else                                                                                                 \
        hipLaunchKernelGGL((k_correlate<L, false>), dim3(unsigned(grid)), dim3(corr_threads(L)), 0, st, segspec, \
                           bank, bank_half, nz, tpb, nb, h, nseg, total, per, grp, plane, codes, code_inv);
    FDAS_SWITCH_LOG2(log2s, CALL)
#undef CALL
    return hipGetLastError();
}

size_t harmsum_scratch_bytes(int nz, int64_t nb, uint32_t cell_cap, uint32_t group_cap) {
    return size_t(group_cap) * sizeof(Group) + size_t(cell_cap) * SUM_STRIDE * sizeof(float) +
           size_t((cell_cap + 1) / 2) * sizeof(uint2) + size_t(nz) * size_t(nb / SC_COLS) * sizeof(uint32_t);
}

hipError_t launch_harmsum(const float *plane, const uint8_t *codes, int nz, int64_t nb, int64_t split, int izc,
                          int nharm_max,
                          const float *thr_host, const uint32_t *code_thr, void *scratch, uint32_t cell_cap,
                          uint32_t group_cap, DevCand *cands, uint32_t *count, uint32_t cap, hipStream_t st) {
    int levels = 0;
    while ((1 << levels) < nharm_max) ++levels;
    if ((1 << levels) != nharm_max || levels > 4) return hipErrorInvalidValue;
    if (nb > (int64_t(1) << 26) || nb % SC_COLS != 0 || nz > 65535) return hipErrorInvalidValue;
    if (split != 0 && 2 * split != nb) return hipErrorInvalidValue;
    Thr thr{};
    ScreenThr T{};
    for (int l = 0; l <= levels; ++l) {
        if (code_thr[l] > 0x8000u) return hipErrorInvalidValue;
        thr.v[l] = thr_host[l];
        T.k[l] = (0x8000u - code_thr[l]) * 0x10001u;
    }
    cell_cap &= ~1u;  // whole blocks
    Group *groups = static_cast<Group *>(scratch);
    float *sums = reinterpret_cast<float *>(groups + group_cap);
    uint2 *blocks = reinterpret_cast<uint2 *>(sums + size_t(cell_cap) * SUM_STRIDE);
    uint32_t *group_map = reinterpret_cast<uint32_t *>(blocks + cell_cap / 2);
    const int64_t rows = SC_TZ, cols = int64_t(SC_WAVE_COLS) * SC_WAVES;
    const dim3 grid1(unsigned((nb + cols - 1) / cols), unsigned((nz + rows - 1) / rows));
    const unsigned grid2 = 2048;
#define CALL(LV)                                                                                                   \
    hipLaunchKernelGGL((k_screen<LV>), grid1, dim3(64 * SC_WAVES), 0, st, codes, nz, nb, izc, T, groups, blocks,    \
                       group_map, count, group_cap, cell_cap);                                                     \
    hipLaunchKernelGGL((k_exact<LV>), dim3(grid2), dim3(256), 0, st, plane, nz, nb, split, izc, blocks, count,      \
                       cell_cap, sums);                                                                            \
    hipLaunchKernelGGL((k_peaks<LV>), dim3(grid2), dim3(256), 0, st, nz, nb, thr, groups, group_map, blocks, sums,  \
                       count, group_cap, cell_cap, cands, cap);
    switch (levels) {
        case 0: CALL(0); break;
        case 1: CALL(1); break;
        case 2: CALL(2); break;
        case 3: CALL(3); break;
        default: CALL(4); break;
    }
#undef CALL
    return hipGetLastError();
}


uint32_t batch_screen_tiles(int64_t nb, int nz) {
    const int64_t cols = int64_t(SC_WAVE_COLS) * SC_WAVES;
    return uint32_t(((nb + cols - 1) / cols) * ((nz + SC_TZ - 1) / SC_TZ));
}

static int harm_levels(int nharm_max) {
    int levels = 0;
    while ((1 << levels) < nharm_max) ++levels;
    return (1 << levels) == nharm_max && levels <= 4 ? levels : -1;
}

hipError_t batch_persistent_workgroups(int log2s, int nharm_max, int *per_cu) {
    const int levels = harm_levels(nharm_max);
    if (levels < 0 || (log2s != 12 && log2s != 13)) return hipErrorInvalidValue;
    hipError_t e = hipErrorInvalidValue;
#define OCC(LS, LV)                                                                                         \
    if (log2s == LS && levels == LV)                                                                        \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void *>(&k_batch<LS, LV>), \
                                                         256, 0);
    OCC(12, 0) OCC(12, 1) OCC(12, 2) OCC(12, 3) OCC(12, 4)
    OCC(13, 0) OCC(13, 1) OCC(13, 2) OCC(13, 3) OCC(13, 4)
#undef OCC
    return e;
}

hipError_t launch_batch_persistent(int log2s, int nharm_max, const BatchTrial *trials, int ntrials,
                                   const uint32_t *tiles, uint32_t ntiles, uint32_t *ctl, int slots,
                                   const float2 *bank, int nz, int tpb, int h, int W, int izc, float code_inv,
                                   const float *thr_host, const uint32_t *code_thr, uint32_t cell_cap,
                                   uint32_t group_cap, uint32_t cand_cap, int workgroups, hipStream_t st) {
    const int levels = harm_levels(nharm_max);
    if (levels < 0 || (log2s != 12 && log2s != 13) || ntrials <= 0 || ntrials > kBatchMaxTrials || slots <= 0 ||
        workgroups <= 0 || nz > 65535)
        return hipErrorInvalidValue;
    BatchArgs a{};
    a.trials = trials;
    a.tiles = tiles;
    a.ctl = ctl;
    a.bank = bank;
    a.ntrials = ntrials;
    a.slots = slots;
    a.nz = nz;
    a.tpb = tpb;
    a.h = h;
    a.W = W;
    a.izc = izc;
    a.ntiles = ntiles;
    a.cell_cap = cell_cap & ~1u;  // whole blocks, as launch_harmsum
    a.group_cap = group_cap;
    a.cand_cap = cand_cap;
    a.code_inv = code_inv;
    for (int l = 0; l <= levels; ++l) {
        if (code_thr[l] > 0x8000u) return hipErrorInvalidValue;
        a.thr.v[l] = thr_host[l];
        a.T.k[l] = (0x8000u - code_thr[l]) * 0x10001u;
    }
#define CALL(LS, LV)                                                                                     \
    if (log2s == LS && levels == LV)                                                                     \
        hipLaunchKernelGGL((k_batch<LS, LV>), dim3(unsigned(workgroups)), dim3(256), 0, st, a);
    CALL(12, 0) CALL(12, 1) CALL(12, 2) CALL(12, 3) CALL(12, 4)
    CALL(13, 0) CALL(13, 1) CALL(13, 2) CALL(13, 3) CALL(13, 4)
#undef CALL
    return hipGetLastError();
}

}  // namespace fdas
