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

// Code of a 2-bin block: the larger of its bins' codes (255 if either is NaN,
// which fmaxf alone would drop).
__device__ __forceinline__ uint8_t block_code(float a, float b, float code_inv) {
    float m = fmaxf(a, b);
    const float sum = a + b;
    if (!(sum == sum)) m = INFINITY;
    return uint8_t(fminf(ceilf(m * code_inv), 255.f));
}

// The codes of the two 2-bin blocks of 4 consecutive bins, as 2 bytes.
__device__ __forceinline__ uint16_t block_codes4(float4 p, float code_inv) {
    return uint16_t(block_code(p.x, p.y, code_inv)) | uint16_t(uint16_t(block_code(p.z, p.w, code_inv)) << 8);
}

}  // namespace fdas
