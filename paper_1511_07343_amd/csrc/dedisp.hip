// De-dispersion (the step before the search, Sec. 1: one time series per
// dispersion-measure trial): the channels of a channel-major 8-bit
// filterbank shifted by their per-DM sample delays and added, in exact
// integer arithmetic.
#include "kernels.hpp"

namespace fdas {

namespace {

constexpr int DD_THREADS = 256;
constexpr int DD_PER = 4;  // consecutive outputs per thread
constexpr int DD_TILE = DD_THREADS * DD_PER;
constexpr int kDdXcds = 8;

// Work item u = (time tile, DM), DM fastest; workgroup i takes item
// (i mod 8) per + i div 8, so the workgroups of one XCD walk consecutive DMs
// of the same time tile and share its channel spans in their L2.
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
    int32_t acc[DD_PER] = {0, 0, 0, 0};
    if (t0 + DD_PER <= nout) {
        for (int c = 0; c < nchan; ++c) {
            const uint8_t *__restrict__ p = fil + int64_t(c) * nsamp + t0 + d[c];
#pragma unroll
            for (int i = 0; i < DD_PER; ++i) acc[i] += int32_t(p[i]);
        }
    } else {
        for (int c = 0; c < nchan; ++c) {
            const uint8_t *__restrict__ p = fil + int64_t(c) * nsamp + t0 + d[c];
#pragma unroll
            for (int i = 0; i < DD_PER; ++i)
                if (t0 + i < nout) acc[i] += int32_t(p[i]);
        }
    }
    float *__restrict__ o = out + int64_t(dm) * nout + t0;
#pragma unroll
    for (int i = 0; i < DD_PER; ++i)
        if (t0 + i < nout) o[i] = float(acc[i]);
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
