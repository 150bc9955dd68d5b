// Device helpers shared by the correlation kernels (FFT and matrix forms).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdas {

constexpr double kLn2 = 0.69314718055994530942;

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

// Screening code of a power: min(255, ceil(P / delta)) with code_inv = 1 / delta,
// never below P / delta (up to one rounding of the product), so integer sums of
// codes bound power sums from above; NaN and huge powers saturate at 255.
__device__ __forceinline__ uint8_t power_code(float pw, float code_inv) {
    return uint8_t(fminf(ceilf(pw * code_inv), 255.f));
}

}  // namespace fdas
