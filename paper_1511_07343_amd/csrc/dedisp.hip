// De-dispersion (the step before the search, Sec. 1: one time series per
// dispersion-measure trial): the channels of a channel-major 8-bit
// filterbank shifted by their per-DM sample delays and added, in exact
// integer arithmetic.
#include "kernels.hpp"

namespace fdas {

namespace {

constexpr int DD_THREADS = 256;
constexpr int DD_PER = 8;  // consecutive outputs per thread
constexpr int DD_TILE = DD_THREADS * DD_PER;
constexpr int kDdXcds = 8;
constexpr int DD_SWAR_CHANNELS = 256;  // 256 x 255 < 2^16: 16-bit partial sums cannot carry

// Work item u = (time tile, DM), DM fastest; workgroup i takes item
// (i mod 8) per + i div 8, so the workgroups of one XCD walk consecutive DMs
// of the same time tile and share its channel spans in their L2.
//
// A thread adds 8 consecutive samples of each channel: it reads the three
// aligned words that cover them, aligns the 8 bytes into two words, and adds
// them as four pairs of 16-bit fields (samples 0/2, 1/3, 4/6, 5/7), flushed
// into 32-bit sums every 256 channels.  Where the three words would run past
// the end of the filterbank the thread reads bytes instead.
__global__ __launch_bounds__(DD_THREADS) void k_dedisperse(const uint8_t *__restrict__ fil, int nchan, int64_t nsamp,
                                                           const int32_t *__restrict__ delays, int ndm, int64_t nout,
                                                           int64_t total, int64_t per, float *__restrict__ out) {
    const int64_t u = int64_t(blockIdx.x % kDdXcds) * per + blockIdx.x / kDdXcds;
    if (u >= total) return;
    const int64_t tile = u / ndm;
    const int dm = int(u - tile * ndm);
    const int64_t t0 = tile * DD_TILE + int64_t(threadIdx.x) * DD_PER;
    if (t0 >= nout) return;
    const int32_t *__restrict__ d = delays + int64_t(dm) * nchan;
    const int64_t fil_bytes = int64_t(nchan) * nsamp;
    uint32_t acc[DD_PER] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool full = t0 + DD_PER <= nout;
    for (int c0 = 0; c0 < nchan; c0 += DD_SWAR_CHANNELS) {
        const int c1 = min(nchan, c0 + DD_SWAR_CHANNELS);
        uint32_t e0 = 0, o0 = 0, e1 = 0, o1 = 0;  // 16-bit pair sums
        for (int c = c0; c < c1; ++c) {
            const int64_t base = int64_t(c) * nsamp + t0 + d[c];
            uint32_t w0, w1;
            const int64_t a = base & ~int64_t(3);
            if (full && a + 12 <= fil_bytes) {
                const uint32_t *__restrict__ q = reinterpret_cast<const uint32_t *>(fil + a);
                const uint32_t q0 = q[0], q1 = q[1], q2 = q[2];
                const uint32_t sh = uint32_t(base - a) * 8u;
                // bytes base .. base + 7 (little endian): funnel shifts of the word pairs
                w0 = sh ? (q0 >> sh) | (q1 << (32u - sh)) : q0;
                w1 = sh ? (q1 >> sh) | (q2 << (32u - sh)) : q1;
            } else {
                w0 = w1 = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (t0 + i < nout) w0 |= uint32_t(fil[base + i]) << (8 * i);
                    if (t0 + 4 + i < nout) w1 |= uint32_t(fil[base + 4 + i]) << (8 * i);
                }
            }
            e0 += w0 & 0x00ff00ffu;
            o0 += (w0 >> 8) & 0x00ff00ffu;
            e1 += w1 & 0x00ff00ffu;
            o1 += (w1 >> 8) & 0x00ff00ffu;
        }
        acc[0] += e0 & 0xffffu;
        acc[1] += o0 & 0xffffu;
        acc[2] += e0 >> 16;
        acc[3] += o0 >> 16;
        acc[4] += e1 & 0xffffu;
        acc[5] += o1 & 0xffffu;
        acc[6] += e1 >> 16;
        acc[7] += o1 >> 16;
    }
    float *__restrict__ o = out + int64_t(dm) * nout + t0;
    if (full && ((reinterpret_cast<uintptr_t>(o) & 15u) == 0)) {
        *reinterpret_cast<float4 *>(o) = make_float4(float(acc[0]), float(acc[1]), float(acc[2]), float(acc[3]));
        *reinterpret_cast<float4 *>(o + 4) = make_float4(float(acc[4]), float(acc[5]), float(acc[6]), float(acc[7]));
    } else {
#pragma unroll
        for (int i = 0; i < DD_PER; ++i)
            if (t0 + i < nout) o[i] = float(acc[i]);
    }
}

}  // namespace

hipError_t launch_dedisperse(const uint8_t *fil, int nchan, int64_t nsamp, const int32_t *delays, int ndm,
                             int64_t nout, float *out, hipStream_t st) {
    if (nchan <= 0 || ndm <= 0 || nout <= 0 || nsamp <= 0) return hipErrorInvalidValue;
    const int64_t tiles = (nout + DD_TILE - 1) / DD_TILE;
    const int64_t total = tiles * ndm;
    const int64_t per = (total + kDdXcds - 1) / kDdXcds;
    const int64_t grid = per * kDdXcds;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dedisperse, dim3(unsigned(grid)), dim3(DD_THREADS), 0, st, fil, nchan, nsamp, delays, ndm,
                       nout, total, per, out);
    return hipGetLastError();
}

}  // namespace fdas
