// Host-side FP64 mathematics of the FDAS library: Fresnel integrals, the
// constant-acceleration template response, a radix-2 FP64 FFT used once per
// plan to move the template bank into the segment domain, and the threshold /
// significance functions.  No device code.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace fdas {

using cd = std::complex<double>;

// F(x) = C(x) + i S(x), C(x) = int_0^x cos(pi t^2 / 2) dt.
cd fresnel(double x);

// A(q, z): Fourier response at offset q bins of a unit tone drifting by z
// bins over the observation (Sec. 2; closed form via Fresnel integrals).
cd accel_response(double q, double z);

// h = ceil(zmax / 2) + 16.
int32_t template_halfwidth(double zmax);

// Taps of one template: conj(A(q, z)) / ||A||, q = -h..h (2h+1 values).
void template_taps(double z, int32_t h, cd *out);
// Half-bin taps: out[q + h] = conj(A(q + 1/2, z)) / norm for q = -h .. h-1 (the
// 2h offsets within h of a point halfway between bins), out[2h] = 0; the norm
// is taken over those 2h taps.
void template_taps_half(double z, int32_t h, cd *out);

// In-place unnormalised FFT, sign -1 forward (e^{-2 pi i n k / n}) or +1.
void fft_inplace(std::vector<cd> &a, int sign);

// log Q(n, S): log of the survival function of a sum of n unit exponentials.
double log_gamma_survival(int32_t n, double s);
// log of the Gaussian upper tail Phi_c(sigma).
double log_normal_tail(double sigma);
// Threshold thr with Q(n, thr) = Phi_c(sigma).
double threshold(double sigma, int32_t n);
// sigma with Phi_c(sigma) = Q(n, power).
double significance(double power, int32_t n);

}  // namespace fdas
