// Host FP64 mathematics: Fresnel integrals, the drifting-tone response
// (template closed form), an FP64 FFT for the plan-time bank transform, and
// the threshold / significance functions.  Written from the mathematics; it
// shares nothing with the test oracle.
#include "host_math.hpp"

#include <cmath>
#include <stdexcept>

namespace fdas {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// (cos(pi x), sin(pi x)) with x reduced mod 2 first.
cd cispi(double x) {
    double r = std::fmod(x, 2.0);
    if (r < 0) r += 2.0;
    // exact values at multiples of 1/2 keep integer offsets exact
    if (r == 0.0) return cd(1.0, 0.0);
    if (r == 0.5) return cd(0.0, 1.0);
    if (r == 1.0) return cd(-1.0, 0.0);
    if (r == 1.5) return cd(0.0, -1.0);
    return cd(std::cos(kPi * r), std::sin(kPi * r));
}

// Power series: F(x) = sum_m (i pi x^2 / 2)^m / m! * x / (2m + 1).
cd fresnel_series(double x) {
    const cd w(0.0, kPi * x * x / 2.0);
    cd term(1.0, 0.0);  // w^m / m!
    cd sum(x, 0.0);
    for (int m = 1; m < 80; ++m) {
        term *= w / double(m);
        cd add = term * (x / double(2 * m + 1));
        sum += add;
        if (std::abs(add) < 1e-18 * std::abs(sum)) break;
    }
    return sum;
}

// Auxiliary G(x) = g(x) + i f(x) for x >= 1.5, defined by
//   F(x) = (1 + i)/2 - G(x) exp(i pi x^2 / 2).
// From F(x) = (1 + i)/2 erf(zeta), zeta = (sqrt(pi)/2)(1 - i) x, and
// erfc(zeta) = exp(-zeta^2)/sqrt(pi) K(zeta) with exp(-zeta^2) = exp(i pi x^2/2):
//   G = (1 + i) / (2 sqrt(pi)) K(zeta),
// K(zeta) = 2 zeta / (b0 - a1/(b1 - a2/(b2 - ...))), b_n = 2 zeta^2 + 1 + 4n,
// a_n = (2n - 1)(2n): the even part of Laplace's continued fraction for erfc,
// evaluated with the modified Lentz method.
cd fresnel_aux(double x) {
    const double sp = std::sqrt(kPi);
    const cd zeta = cd(sp / 2.0 * x, -sp / 2.0 * x);
    const cd two_z2(0.0, -kPi * x * x);  // 2 zeta^2
    const double tiny = 1e-300;
    cd b = two_z2 + 1.0;
    cd f = b;
    if (std::abs(f) == 0.0) f = tiny;
    cd C = f, D = 0.0;
    for (int n = 1; n < 100000; ++n) {
        const double an = -double(2 * n - 1) * double(2 * n);
        b += 4.0;
        D = b + an * D;
        if (std::abs(D) == 0.0) D = tiny;
        D = 1.0 / D;
        C = b + an / C;
        if (std::abs(C) == 0.0) C = tiny;
        const cd delta = C * D;
        f *= delta;
        if (std::abs(delta - 1.0) < 1e-16) break;
    }
    const cd K = 2.0 * zeta / f;
    return cd(1.0, 1.0) / (2.0 * sp) * K;
}

}  // namespace

cd fresnel(double x) {
    const double ax = std::fabs(x);
    cd r;
    if (ax < 1.5) {
        r = fresnel_series(ax);
    } else {
        r = cd(0.5, 0.5) - fresnel_aux(ax) * cispi(ax * ax / 2.0);
    }
    return x < 0 ? -r : r;
}

cd accel_response(double q, double z) {
    if (z == 0.0) {
        if (q == std::nearbyint(q)) return q == 0.0 ? cd(1.0, 0.0) : cd(0.0, 0.0);
        const double s = std::sin(kPi * q) / (kPi * q);
        return cispi(q) * s;
    }
    if (z < 0.0) return std::conj(accel_response(-q, -z));
    // A(q, z) = A_s(p, z), p = q - z/2:
    //   A_s = exp(-i pi p^2 / z) / sqrt(2z) [F(Z) - F(Y)], Y = p sqrt(2/z), Z = Y + sqrt(2z).
    const double p = q - z / 2.0;
    const double s = std::sqrt(2.0 / z);
    const double Y = p * s, Zv = (p + z) * s;
    const double pre = 1.0 / std::sqrt(2.0 * z);
    // exp(i pi (Z^2 - Y^2) / 2) = exp(i pi (2p + z)) = exp(2 pi i q)
    if (Y >= 1.5) {
        // both ends on the positive tail: the (1+i)/2 constants cancel exactly
        return pre * (fresnel_aux(Y) - fresnel_aux(Zv) * cispi(2.0 * q));
    }
    if (Zv <= -1.5) {
        return pre * (fresnel_aux(-Zv) * cispi(2.0 * q) - fresnel_aux(-Y));
    }
    return pre * cispi(-(p * p / z)) * (fresnel(Zv) - fresnel(Y));
}

int32_t template_halfwidth(double zmax) { return int32_t(std::ceil(zmax / 2.0)) + 16; }

void template_taps(double z, int32_t h, cd *out) {
    double e = 0.0;
    for (int32_t q = -h; q <= h; ++q) {
        const cd a = accel_response(double(q), z);
        out[q + h] = std::conj(a);
        e += std::norm(a);
    }
    const double inv = 1.0 / std::sqrt(e);
    for (int32_t i = 0; i < 2 * h + 1; ++i) out[i] *= inv;
}

void template_taps_half(double z, int32_t h, cd *out) {
    double e = 0.0;
    for (int32_t q = -h; q < h; ++q) {
        const cd a = accel_response(double(q) + 0.5, z);
        out[q + h] = std::conj(a);
        e += std::norm(a);
    }
    out[2 * h] = cd(0.0, 0.0);
    const double inv = 1.0 / std::sqrt(e);
    for (int32_t i = 0; i < 2 * h; ++i) out[i] *= inv;
}

void fft_inplace(std::vector<cd> &a, int sign) {
    const size_t n = a.size();
    if (n == 0 || (n & (n - 1))) throw std::invalid_argument("fft length must be a power of two");
    for (size_t i = 1, j = 0; i < n; ++i) {  // bit reversal
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    std::vector<cd> w(n / 2);
    for (size_t k = 0; k < n / 2; ++k) w[k] = cispi(double(sign) * 2.0 * double(k) / double(n));
    for (size_t len = 2; len <= n; len <<= 1) {
        const size_t step = n / len;
        for (size_t i = 0; i < n; i += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                const cd u = a[i + k];
                const cd v = a[i + k + len / 2] * w[k * step];
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

double log_gamma_survival(int32_t n, double s) {
    if (s <= 0.0) return 0.0;
    // log sum_{i<n} s^i / i!, by log-sum-exp
    double mx = -INFINITY;
    std::vector<double> t(n);
    for (int32_t i = 0; i < n; ++i) {
        t[i] = double(i) * std::log(s) - std::lgamma(double(i) + 1.0);
        if (t[i] > mx) mx = t[i];
    }
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) acc += std::exp(t[i] - mx);
    return -s + mx + std::log(acc);
}

double log_normal_tail(double sigma) {
    if (sigma < 30.0) return std::log(0.5 * std::erfc(sigma / std::sqrt(2.0)));
    // asymptotic series of the Mills ratio
    const double s2 = 1.0 / (sigma * sigma);
    const double series = 1.0 - s2 + 3.0 * s2 * s2 - 15.0 * s2 * s2 * s2 + 105.0 * s2 * s2 * s2 * s2;
    return -0.5 * sigma * sigma - std::log(sigma) - 0.5 * std::log(2.0 * kPi) + std::log(series);
}

double threshold(double sigma, int32_t n) {
    const double target = log_normal_tail(sigma);
    double lo = 0.0, hi = 16.0;
    while (log_gamma_survival(n, hi) > target) hi *= 2.0;
    for (int it = 0; it < 400 && hi - lo > 1e-15 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (log_gamma_survival(n, mid) > target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double significance(double power, int32_t n) {
    const double target = log_gamma_survival(n, power);
    double lo = -40.0, hi = 40.0;
    if (log_normal_tail(lo) < target) return lo;
    while (log_normal_tail(hi) > target) hi *= 2.0;
    for (int it = 0; it < 400 && hi - lo > 1e-13 * std::fmax(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (log_normal_tail(mid) > target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

}  // namespace fdas
