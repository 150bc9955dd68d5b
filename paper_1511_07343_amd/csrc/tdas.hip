// Time-domain resampling acceleration search (the other method of Sec. 1:
// resample the series for each acceleration trial, then one long DFT each).
// The DFT, the block medians and the harmonic sums are the FDAS kernels; this
// file holds the resampling, the normalised powers with their screening codes
// and the drift of the reported candidates.
#include "device_common.hpp"
#include "kernels.hpp"

#include <cmath>

namespace fdas {

namespace {

// y[m] = x at position s_m = N (v_m + 1/2), v_m = 2 tau_m / (1 + sqrt(1 + 2 alpha tau_m)),
// tau_m = m / N - 1/2: the time axis on which a tone drifting by alpha
// (relative to its mean frequency) keeps one frequency.  Linear interpolation
// between the neighbouring samples (x[N] = 0), zero outside the series.  The
// position is formed in FP64 (it needs ~24 bits of integer part plus the
// fraction).
__global__ __launch_bounds__(256) void k_td_resample(const float *__restrict__ x, int64_t n, double alpha,
                                                     float *__restrict__ y) {
    const double inv_n = 1.0 / double(n);
    for (int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; m < n; m += int64_t(gridDim.x) * blockDim.x) {
        const double tau = double(m) * inv_n - 0.5;
        const double v = 2.0 * tau / (1.0 + sqrt(1.0 + 2.0 * alpha * tau));
        const double s = double(n) * (v + 0.5);
        const double fl = floor(s);
        const int64_t i = int64_t(fl);
        float out = 0.f;
        if (i >= 0 && i <= n - 1) {
            const double f = s - fl;
            const double a = double(x[i]);
            const double b = i + 1 < n ? double(x[i + 1]) : 0.0;
            out = float(a * (1.0 - f) + b * f);
        }
        y[m] = out;
    }
}

// P[k] = |X[k]|^2 ln2 / m(k) for 4 consecutive bins per thread, and the
// screening codes of their two 2-bin blocks.  nb % 4 == 0.
__global__ __launch_bounds__(256) void k_td_power(const float2 *__restrict__ X, const double *__restrict__ med, int W,
                                                  int64_t nb, float *__restrict__ row, uint8_t *__restrict__ qrow,
                                                  float code_inv) {
    const int64_t nblk = (nb + W - 1) / W;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; 4 * c < nb;
         c += int64_t(gridDim.x) * blockDim.x) {
        float p[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t k = 4 * c + i;
            const float2 v = X[k];
            const double m = median_curve(med, nblk, W, nb, k);
            const double scale = m > 0.0 ? kLn2 / m : 0.0;
            p[i] = float((double(v.x) * double(v.x) + double(v.y) * double(v.y)) * scale);
        }
        const float4 p4 = make_float4(p[0], p[1], p[2], p[3]);
        *reinterpret_cast<float4 *>(row + 4 * c) = p4;
        *reinterpret_cast<uint16_t *>(qrow + 2 * c) = block_codes4(p4, code_inv);
    }
}

// Candidate drift of a time-domain search: z = alpha(iz) r, alpha(iz) =
// -alpha_max + iz d (0 for a single trial).
__global__ __launch_bounds__(256) void k_td_drift(const uint32_t *__restrict__ count, uint32_t cap, double alpha_max,
                                                  double d, int single, fdas_cand *__restrict__ cands) {
    // -alpha_max + d iz with two roundings, as the trials are formed (a fused
    // multiply-add would round once and can differ in the last bit)
#pragma clang fp contract(off)
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double a = single ? 0.0 : -alpha_max + d * double(cands[i].iz);
        cands[i].z = a * cands[i].r;
    }
}

unsigned grid_for(int64_t items) {
    const int64_t g = (items + 255) / 256;
    return unsigned(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_td_resample(const float *x, int64_t nsamp, double alpha, float *y, hipStream_t st) {
    if (nsamp <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_td_resample, dim3(grid_for(nsamp)), dim3(256), 0, st, x, nsamp, alpha, y);
    return hipGetLastError();
}

hipError_t launch_td_power(const float2 *X, const double *med, int W, int64_t nb, float *row, uint8_t *qrow,
                           float code_inv, hipStream_t st) {
    if (nb <= 0 || nb % 4 != 0 || W <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_td_power, dim3(grid_for(nb / 4)), dim3(256), 0, st, X, med, W, nb, row, qrow, code_inv);
    return hipGetLastError();
}

hipError_t launch_td_drift(const uint32_t *count, uint32_t cap, double alpha_max, int nalpha, fdas_cand *cands,
                           hipStream_t st) {
    if (cap == 0) return hipSuccess;
    const double d = nalpha > 1 ? 2.0 * alpha_max / double(nalpha - 1) : 0.0;
    hipLaunchKernelGGL(k_td_drift, dim3(grid_for(cap)), dim3(256), 0, st, count, cap, alpha_max, d, nalpha == 1 ? 1 : 0,
                       cands);
    return hipGetLastError();
}

}  // namespace fdas
