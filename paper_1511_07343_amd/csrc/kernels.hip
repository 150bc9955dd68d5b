// FDAS device kernels for gfx950 (CDNA4).  Steps follow Sec. 4 of Dimoudi &
// Armour (arXiv:1511.07343): real-to-complex DFT (step 2), overlapped segments
// and their DFTs (steps 3-4, the overlap copy folded into the segment loader),
// complex multiply-scale by every template (step 5), inverse DFT (step 6) and
// power with edge removal (step 7) fused into one kernel; then harmonic sums,
// thresholds and local maxima on the resulting f-fdot plane.
#include "fft_wg.hpp"
#include "kernels.hpp"

#include <cmath>

namespace fdas {

namespace {

constexpr double kLn2 = 0.69314718055994530942;

// Threads per workgroup for a transform of 2^log2s points.
constexpr int fft_threads(int log2s) {
    return log2s >= 12 ? 256 : log2s == 11 ? 128 : log2s >= 8 ? 64 : 32;
}

// Threads per workgroup of the fused correlation kernel.
constexpr int corr_threads(int log2s) { return fft_threads(log2s); }

// 8 XCDs on MI355X; workgroups are dispatched to XCDs round-robin by index.
constexpr int kXcds = 8;

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
    const int64_t n2 = blockIdx.x;
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
    const int64_t k1 = blockIdx.x;
    Twiddles<Sh, -1> tw;
    tw.init(t);
    float2 v[Sh::R];
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) v[m] = work[(k1 << LOG2M2) + t + Sh::NT * m];
    fft_wg<Sh, -1>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) Z[k1 + (int64_t(t + Sh::NT * m) << log2m1)] = v[m];
}

// ------------------------------------------------------ medians of |X|^2
// Ascending bitonic sort of W (power of two) floats in LDS.
__device__ void bitonic_sort_lds(float *s, int W) {
    const int t = threadIdx.x, nt = blockDim.x;
    for (int size = 2; size <= W; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = t; i < (W >> 1); i += nt) {
                const int lo = 2 * stride * (i / stride) + (i % stride);
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const float a = s[lo], b = s[hi];
                if ((a > b) == asc) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
        }
    }
    __syncthreads();
}

constexpr int kMedThreads = 256;
constexpr int kMaxW = 8192;

// Median of the sorted valid prefix of length w (mean of the middle pair for
// even w), in FP64.
__device__ __forceinline__ double median_sorted(const float *s, int w) {
    return (w & 1) ? double(s[w >> 1]) : 0.5 * (double(s[(w >> 1) - 1]) + double(s[w >> 1]));
}

// One workgroup per block of W bins: X[k] from Z[k] and Z[M - k], then the
// block's median power.
__global__ __launch_bounds__(kMedThreads) void k_unpack_median(const float2 *__restrict__ Z,
                                                               int64_t M, float2 *__restrict__ X,
                                                               double *__restrict__ med, int W) {
    __shared__ float s[kMaxW];
    const int t = threadIdx.x;
    const int64_t b0 = int64_t(blockIdx.x) * W;
    const int w = int(min(int64_t(W), M - b0));
    const double inv_n = 1.0 / double(2 * M);
    for (int i = t; i < W; i += kMedThreads) {
        float p = INFINITY;
        if (i < w) {
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
            p = cnorm(x);
        }
        s[i] = p;
    }
    bitonic_sort_lds(s, W);
    if (t == 0) med[blockIdx.x] = median_sorted(s, w);
}

__global__ __launch_bounds__(kMedThreads) void k_median(const float2 *__restrict__ X, int64_t nb,
                                                        double *__restrict__ med, int W) {
    __shared__ float s[kMaxW];
    const int t = threadIdx.x;
    const int64_t b0 = int64_t(blockIdx.x) * W;
    const int w = int(min(int64_t(W), nb - b0));
    for (int i = t; i < W; i += kMedThreads) s[i] = i < w ? cnorm(X[b0 + i]) : INFINITY;
    bitonic_sort_lds(s, W);
    if (t == 0) med[blockIdx.x] = median_sorted(s, w);
}

// m(k): block medians joined linearly between block centres, flat outside.
__device__ __forceinline__ double median_curve(const double *__restrict__ med, int64_t nblk, int W,
                                               int64_t nb, int64_t g) {
    const double c0 = 0.5 * double(min(int64_t(W), nb) - 1);
    const int64_t wl = nb - (nblk - 1) * int64_t(W);
    const double cl = double((nblk - 1) * int64_t(W)) + 0.5 * double(wl - 1);
    const double x = double(g);
    if (x <= c0 || nblk == 1) return med[0];
    if (x >= cl) return med[nblk - 1];
    const int64_t b = int64_t(floor((x - c0) / double(W)));
    const double cb = c0 + double(b) * double(W);
    const double cb1 = (b + 1 == nblk - 1) ? cl : cb + double(W);
    return med[b] + (med[b + 1] - med[b]) * ((x - cb) / (cb1 - cb));
}

// -------------------------------------------------------- segment DFTs
template <int LOG2S>
__global__ __launch_bounds__(fft_threads(LOG2S)) void k_segfft(const float2 *__restrict__ X,
                                                               const double *__restrict__ med,
                                                               int W, int64_t nb, int h,
                                                               float2 *__restrict__ segspec) {
    using Sh = FftShape<LOG2S, fft_threads(LOG2S)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    const int64_t s = blockIdx.x;
    const int64_t L = Sh::S - 2 * h;
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
    fft_wg<Sh, -1>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < Sh::R; ++m) segspec[s * Sh::S + t + Sh::NT * m] = v[m];
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
// Work item u = (template block tb, segment s), tb-major.  Workgroup i runs
// item u = (i mod 8) * per + i div 8, so each XCD walks a contiguous range of
// template blocks over all segments and keeps its templates in its own L2.
template <int LOG2S>
__global__ __launch_bounds__(corr_threads(LOG2S), 2) void k_correlate(
    const float2 *__restrict__ segspec, const float2 *__restrict__ bank, int nz, int tpb, int64_t nb,
    int h, int64_t nseg, int64_t total, int64_t per, float *__restrict__ plane) {
    using Sh = FftShape<LOG2S, corr_threads(LOG2S)>;
    __shared__ float2 lds[Sh::LDS_FLOAT2];
    const int t = threadIdx.x;
    const int64_t u = int64_t(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    if (u >= total) return;
    const int64_t tb = u / nseg;
    const int64_t s = u - tb * nseg;
    const int64_t L = Sh::S - 2 * h;
    const int iz0 = int(tb) * tpb;
    const int iz1 = min(nz, iz0 + tpb);

    Twiddles<Sh, +1> tw;
    tw.init(t);
    // The segment spectrum is re-read per template (from L2: consecutive
    // workgroups of an XCD share it); keeping it in registers would spill.
    const float2 *__restrict__ sp = segspec + s * Sh::S;

    const int64_t kbase = s * L - h;  // plane column of segment point n is kbase + n
    // columns [kbase + h, kend) of the plane come from this segment
    const int nend = int(min(int64_t(Sh::S - h), nb - kbase));
    for (int iz = iz0; iz < iz1; ++iz) {
        // Keep the per-point offsets inside the loop: hoisting the 32 addresses
        // of each operand out of it would cost more registers than recomputing.
        int to = t;
        asm volatile("" : "+v"(to));
        const float2 *__restrict__ bz = bank + int64_t(iz) * Sh::S;
        float2 v[Sh::R];
#pragma unroll
        for (int m = 0; m < Sh::R; ++m) v[m] = cmul(sp[to + Sh::NT * m], bz[to + Sh::NT * m]);
        fft_wg<Sh, +1>(v, lds, tw, t);
        float *__restrict__ row = plane + int64_t(iz) * nb + kbase;
#pragma unroll
        for (int m = 0; m < Sh::R; ++m) {
            const int n = to + Sh::NT * m;
            if (n >= h && n < nend) row[n] = cnorm(v[m]);
        }
    }
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
__device__ __forceinline__ int frac_row(int izc, int d, int j) {
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
template <int LEVELS>
__device__ __forceinline__ void cell_sums(const float *__restrict__ P, int64_t nb, int izc, int iz, int k,
                                          float (&s)[5]) {
    float v[17];
    v[0] = 0.f;
    const int d = iz - izc;
    static_for<1, 17>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (frac_used<LEVELS>(j)) v[j] = P[int64_t(frac_row(izc, d, j)) * nb + ((j * k + 8) >> 4)];
        else v[j] = 0.f;
    });
    nested_sums<LEVELS>(v, s);
}

// Append the lanes with `pred` to a list through one atomic per wave.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t *__restrict__ counter, int lane, bool &taken) {
    const uint64_t mask = __ballot(pred);
    taken = false;
    if (!mask) return 0;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, uint32_t(__popcll(mask)));
    base = __shfl(base, leader);
    taken = pred;
    return base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
}

// Pass 1: sums of every cell, thresholds, and a list of the cells that reach
// the threshold of any level ("hits": column, row, level mask).
// A wave owns columns k = k0 + lane + 64 i (i < HS_C) and walks HS_TZ
// consecutive rows.  With kl = k0 + lane, c_j(kl + 64 i) = c_j(kl) + 4 j i:
// one base address per fraction and compile-time offsets.  The HS_C values of
// fraction j stay in registers and are reloaded only when r_j moves between
// consecutive rows (a wave-uniform test).
constexpr int HS_C = 4;
constexpr int HS_TZ = 16;
constexpr int HS_WAVES = 4;

struct Hit {
    int32_t k;
    uint32_t iz_mask;  // row in bits 0..15, level mask in bits 16..20
};

template <int LEVELS>
__global__ __launch_bounds__(64 * HS_WAVES) void k_hits(const float *__restrict__ P, int nz, int64_t nb, int izc,
                                                        Thr thr, Hit *__restrict__ hits,
                                                        uint32_t *__restrict__ hit_count, uint32_t hit_cap) {
    // nb is a multiple of 64 * HS_C (checked at launch): a wave's columns are
    // all inside the plane or all outside it.
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t k0 = (int64_t(blockIdx.x) * HS_WAVES + wave) * (64 * HS_C);
    if (k0 >= nb) return;
    const int iz0 = blockIdx.y * HS_TZ;
    const int iz1 = min(nz, iz0 + HS_TZ);
    const int kl = int(k0) + lane;
    float val[17][HS_C];
    for (int iz = iz0; iz < iz1; ++iz) {
        const int d = iz - izc;
        int klo = kl;  // recomputing the column bases per row is cheaper than holding them
        asm volatile("" : "+v"(klo));
        static_for<1, 17>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (frac_used<LEVELS>(j)) {
                const int row = frac_row(izc, d, j);
                if (iz == iz0 || row != frac_row(izc, d - 1, j)) {
                    const float *__restrict__ src = P + int64_t(row) * nb + ((j * klo + 8) >> 4);
#pragma unroll
                    for (int i = 0; i < HS_C; ++i) val[j][i] = src[4 * j * i];
                }
            }
        });
#pragma unroll
        for (int i = 0; i < HS_C; ++i) {
            float v[17];
            v[0] = 0.f;
#pragma unroll
            for (int j = 1; j < 17; ++j) v[j] = val[j][i];
            float sm[5];
            nested_sums<LEVELS>(v, sm);
            uint32_t mask = 0;
#pragma unroll
            for (int l = 0; l <= LEVELS; ++l) mask |= (sm[l] >= thr.v[l] ? 1u : 0u) << l;
            bool taken;
            const uint32_t slot = wave_append(mask != 0, hit_count, lane, taken);
            if (taken && slot < hit_cap) hits[slot] = Hit{kl + 64 * i, uint32_t(iz) | (mask << 16)};
        }
    }
}

// Pass 2, one hit per lane: recompute the hit cell's sums and its 8
// neighbours' (same loads, same order as pass 1) and keep, for every level in
// the mask, a 3x3 local maximum: strictly greater than the neighbours earlier
// in row-major (iz, k) order, at least equal to the later ones; neighbours
// outside the plane are ignored.
template <int LEVELS>
__global__ __launch_bounds__(256) void k_peaks(const float *__restrict__ P, int nz, int64_t nb, int izc,
                                               const Hit *__restrict__ hits, const uint32_t *__restrict__ hit_count,
                                               uint32_t hit_cap, DevCand *__restrict__ cands,
                                               uint32_t *__restrict__ count, uint32_t cap) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = min(*hit_count, hit_cap);
    const uint32_t stride = gridDim.x * blockDim.x;
    // whole waves iterate together so that the appends stay wave-wide
    for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
        const uint32_t h = base + lane;
        const bool valid = h < n;
        int k = 0, iz = 0;
        uint32_t mask = 0;
        if (valid) {
            const Hit r = hits[h];
            k = r.k;
            iz = int(r.iz_mask & 0xffffu);
            mask = r.iz_mask >> 16;
        }
        float s[5];
        cell_sums<LEVELS>(P, nb, izc, iz, k, s);
#pragma unroll 1
        for (int di = -1; di <= 1; ++di) {
            const int iz2 = iz + di;
            const bool rin = iz2 >= 0 && iz2 < nz;
#pragma unroll
            for (int dk = -1; dk <= 1; ++dk) {
                if (di == 0 && dk == 0) continue;
                const int k2 = k + dk;
                const bool in = valid && rin && k2 >= 0 && int64_t(k2) < nb;
                float s2[5];
                cell_sums<LEVELS>(P, nb, izc, in ? iz2 : iz, in ? k2 : k, s2);
                const bool earlier = di < 0 || (di == 0 && dk < 0);
#pragma unroll
                for (int l = 0; l <= LEVELS; ++l) {
                    const bool beaten = earlier ? !(s[l] > s2[l]) : !(s[l] >= s2[l]);
                    if (in && beaten) mask &= ~(1u << l);
                }
            }
        }
#pragma unroll
        for (int l = 0; l <= LEVELS; ++l) {
            bool taken;
            const uint32_t slot = wave_append(valid && ((mask >> l) & 1u), count, lane, taken);
            if (taken && slot < cap) cands[slot] = DevCand{k, iz, 1 << l, s[l]};
        }
    }
}

// A hit list that overflowed makes the candidate list incomplete: raise a flag
// the host turns into OVERFLOW.
__global__ void k_flag_hit_overflow(const uint32_t *__restrict__ hit_count, uint32_t hit_cap,
                                    uint32_t *__restrict__ flag) {
    if (threadIdx.x == 0 && *hit_count > hit_cap) *flag = 1u;
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
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
    const int l1 = (log2m + 1) / 2, l2 = log2m / 2;
    const unsigned ncols = 1u << l2, nrows = 1u << l1;
#define CALL(L) hipLaunchKernelGGL((k_r2c_cols<L>), dim3(ncols), dim3(fft_threads(L)), 0, st, z, work, l2);
    FDAS_SWITCH_LOG2(l1, CALL)
#undef CALL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define CALL(L) hipLaunchKernelGGL((k_r2c_rows<L>), dim3(nrows), dim3(fft_threads(L)), 0, st, work, Z, l1);
    FDAS_SWITCH_LOG2(l2, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_unpack_median(const float2 *Z, int64_t nsamp, float2 *X, double *med, int W, hipStream_t st) {
    const int64_t M = nsamp / 2;
    if (W < 2 || W > kMaxW || (W & (W - 1))) return hipErrorInvalidValue;
    const int64_t nblk = (M + W - 1) / W;
    hipLaunchKernelGGL(k_unpack_median, dim3(unsigned(nblk)), dim3(kMedThreads), 0, st, Z, M, X, med, W);
    return hipGetLastError();
}

hipError_t launch_median(const float2 *X, int64_t nb, double *med, int W, hipStream_t st) {
    if (W < 2 || W > kMaxW || (W & (W - 1))) return hipErrorInvalidValue;
    const int64_t nblk = (nb + W - 1) / W;
    hipLaunchKernelGGL(k_median, dim3(unsigned(nblk)), dim3(kMedThreads), 0, st, X, nb, med, W);
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

hipError_t launch_correlate(const float2 *segspec, const float2 *bank, int nz, int tpb, int64_t nb,
                            int log2s, int h, int64_t nseg, float *plane, hipStream_t st) {
    if (nseg <= 0 || nz <= 0) return hipSuccess;
    if (tpb <= 0) return hipErrorInvalidValue;
    const int64_t nzb = (nz + tpb - 1) / tpb;
    const int64_t total = nzb * nseg;
    const int64_t per = (total + kXcds - 1) / kXcds;
    const int64_t grid = per * kXcds;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
#define CALL(L)                                                                                       \
    hipLaunchKernelGGL((k_correlate<L>), dim3(unsigned(grid)), dim3(corr_threads(L)), 0, st, segspec, bank, \
                       nz, tpb, nb, h, nseg, total, per, plane);
    FDAS_SWITCH_LOG2(log2s, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_harmsum(const float *plane, int nz, int64_t nb, int izc, int nharm_max, const float *thr_host,
                          void *hit_buf, uint32_t hit_cap, DevCand *cands, uint32_t *count, uint32_t cap,
                          hipStream_t st) {
    int levels = 0;
    while ((1 << levels) < nharm_max) ++levels;
    if ((1 << levels) != nharm_max || levels > 4) return hipErrorInvalidValue;
    if (nb > (int64_t(1) << 26) || nb % (64 * HS_C) != 0 || nz > 65535) return hipErrorInvalidValue;
    Thr thr{};
    for (int l = 0; l <= levels; ++l) thr.v[l] = thr_host[l];
    Hit *hits = static_cast<Hit *>(hit_buf);
    uint32_t *hit_count = count + 1;  // the counter pair is zeroed by the caller
    const int64_t cols = 64 * HS_C * HS_WAVES;
    const dim3 grid1(unsigned((nb + cols - 1) / cols), unsigned((nz + HS_TZ - 1) / HS_TZ));
    const unsigned grid2 = 2048;
#define CALL(LV)                                                                                                \
    hipLaunchKernelGGL((k_hits<LV>), grid1, dim3(64 * HS_WAVES), 0, st, plane, nz, nb, izc, thr, hits, hit_count, \
                       hit_cap);                                                                               \
    hipLaunchKernelGGL((k_peaks<LV>), dim3(grid2), dim3(256), 0, st, plane, nz, nb, izc, hits, hit_count, hit_cap,  \
                       cands, count, cap);
    switch (levels) {
        case 0: CALL(0); break;
        case 1: CALL(1); break;
        case 2: CALL(2); break;
        case 3: CALL(3); break;
        default: CALL(4); break;
    }
#undef CALL
    hipLaunchKernelGGL(k_flag_hit_overflow, dim3(1), dim3(64), 0, st, hit_count, hit_cap, count + 2);
    return hipGetLastError();
}

size_t hit_record_bytes() { return sizeof(Hit); }

}  // namespace fdas
