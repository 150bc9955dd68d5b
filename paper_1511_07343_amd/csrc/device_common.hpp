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
    // W is a power of two, so dividing by it is the exact multiply by 1 / W;
    // the last interval (to the centre of a partial last block) is shorter,
    // and its reciprocal width does not depend on g (computed once per
    // thread when inlined in a loop)
    const double inv_w = 1.0 / double(W);
    const double inv_last = 1.0 / (cl - (c0 + double(nblk - 2) * double(W)));
    const int64_t b = int64_t(floor((x - c0) * inv_w));
    const double cb = c0 + double(b) * double(W);
    const double f = (x - cb) * (b + 1 == nblk - 1 ? inv_last : inv_w);
    return med[b] + (med[b + 1] - med[b]) * f;
}

// Screening code of a power: min(255, ceil(P / delta)) with code_inv = 1 / delta,
// never below P / delta (up to one rounding of the product), so integer sums of
// codes bound power sums from above; NaN and huge powers saturate at 255.
__device__ __forceinline__ uint8_t power_code(float pw, float code_inv) {
    return uint8_t(fminf(ceilf(pw * code_inv), 255.f));
}

// Code of a 2-bin block: the larger of its bins' codes, 255 if either is NaN.
// Powers are non-negative (or NaN), and non-negative floats, with NaN above
// +inf, order as their unsigned bit patterns, so one integer maximum picks
// the larger power and keeps a NaN (fmaxf alone would drop it).
__device__ __forceinline__ uint8_t block_code(float a, float b, float code_inv) {
    const float m = __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
    return uint8_t(fminf(ceilf(m * code_inv), 255.f));
}

// The codes of the two 2-bin blocks of 4 consecutive bins, as 2 bytes.
__device__ __forceinline__ uint16_t block_codes4(float4 p, float code_inv) {
    return uint16_t(block_code(p.x, p.y, code_inv)) | uint16_t(uint16_t(block_code(p.z, p.w, code_inv)) << 8);
}

// Single-trial significance in FP64: log Q(n, s) of a sum of n unit-mean
// exponential powers, log Phi_c of the Gaussian tail, and sigma from them.
__device__ inline double log_gamma_survival_d(int n, double s) {
    if (s <= 0.0) return 0.0;
    const double ls = log(s);
    double mx = -INFINITY, lf = 0.0;
    for (int i = 0; i < n; ++i) {  // log(i!) accumulated exactly enough for i <= 16
        if (i > 0) lf += log(double(i));
        mx = fmax(mx, double(i) * ls - lf);
    }
    double acc = 0.0;
    lf = 0.0;
    for (int i = 0; i < n; ++i) {
        if (i > 0) lf += log(double(i));
        acc += exp(double(i) * ls - lf - mx);
    }
    return -s + mx + log(acc);
}

__device__ inline double log_normal_tail_d(double sg) {
    if (sg < 30.0) return log(0.5 * erfc(sg * 0.70710678118654752440));
    const double s2 = 1.0 / (sg * sg);
    const double series = 1.0 - s2 + 3.0 * s2 * s2 - 15.0 * s2 * s2 * s2 + 105.0 * s2 * s2 * s2 * s2;
    return -0.5 * sg * sg - log(sg) - 0.91893853320467274178 + log(series);
}

// sigma with Phi_c(sigma) = Q(n, power): Newton's method on
// f(sigma) = log Phi_c(sigma) - log Q, with f' = -phi(sigma) / Phi_c(sigma)
// (f is decreasing and concave), inside a bracket that falls back to
// bisection whenever a Newton step leaves it.
__device__ inline double significance_d(double power, int n) {
    const double target = log_gamma_survival_d(n, power);
    double lo = -40.0, hi = 40.0;
    if (log_normal_tail_d(lo) < target) return lo;
    while (log_normal_tail_d(hi) > target && hi < 1e9) hi *= 2.0;
    // start from the tail asymptote log Phi_c(x) ~ -x^2/2 - log(x sqrt(2 pi))
    double x = sqrt(fmax(-2.0 * target, 1.0));
    x = fmin(fmax(x, lo), hi);
    for (int it = 0; it < 100; ++it) {
        const double lt = log_normal_tail_d(x);
        const double f = lt - target;
        if (f > 0.0) lo = x; else hi = x;
        const double dlog = -exp(-0.5 * x * x - 0.91893853320467274178 - lt);  // d/dx log Phi_c
        double nx = x - f / dlog;
        if (fabs(nx - x) <= 1e-12 * fmax(1.0, fabs(x))) {
            x = nx;
            break;
        }
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        x = nx;
        if (hi - lo <= 1e-12 * fmax(1.0, fabs(hi))) break;
    }
    return x;
}

}  // namespace fdas
