// Fourier interpolation of the correlation off the (k, z) grid and the
// refinement of candidates by a pattern search over fractional (r, z).  This
// extends the paper's method: the drifting-tone response of Sec. 2 (the
// template of Eq. (1)) is evaluated at any offset and drift instead of the
// integer offsets of the template bank.  Everything is FP64 except the
// spectrum, which is read in FP32 as the search holds it.
#include "device_common.hpp"
#include "fresnel_coeffs.hpp"
#include "kernels.hpp"

#include <cmath>
#include <mutex>

namespace fdas {

namespace {

constexpr double kPiD = 3.14159265358979323846264338327950288;
// A workgroup refines one record at a time; its 16 waves share the record's
// (point, harmonic) pairs, so that a few hundred records fill the GPU.
constexpr int RF_THREADS = 1024;
constexpr int RF_POINT_THREADS = 256;  // workgroup of the point evaluator
constexpr int RF_POINTS = 8;    // neighbours per search level
constexpr int RF_MAX_NH = 16;

struct c64 {
    double re, im;
};
__device__ __forceinline__ c64 cadd(c64 a, c64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c64 csub(c64 a, c64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c64 cmul(c64 a, c64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c64 cscale(c64 a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ double cnorm2(c64 a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ c64 cinv(c64 a) {
    const double d = 1.0 / cnorm2(a);
    return {a.re * d, -a.im * d};
}
__device__ __forceinline__ c64 cdiv(c64 a, c64 b) { return cmul(a, cinv(b)); }

// exp(i pi x), with x reduced to [0, 2) first and exact values at the
// multiples of 1/2 (so that integer offsets give exact results).
__device__ c64 cis_pi(double x) {
    const double r = x - 2.0 * floor(0.5 * x);
    if (r == 0.0) return {1.0, 0.0};
    if (r == 0.5) return {0.0, 1.0};
    if (r == 1.0) return {-1.0, 0.0};
    if (r == 1.5) return {0.0, -1.0};
    double s, c;
    sincospi(r, &s, &c);
    return {c, s};
}

// Fresnel integrals F(x) = C(x) + i S(x), C(x) = int_0^x cos(pi t^2 / 2) dt,
// from the polynomial data of fresnel_coeffs.hpp (written by
// gen_fresnel_coeffs.py): the power series for |x| < 1, and for x >= 1 the
// auxiliary functions f, g of F(x) = (1 + i)/2 - (g + i f) exp(i pi x^2 / 2)
// as Chebyshev expansions in u = 1 / x^2 of pi x f and pi^2 x^3 g.  No loop
// with a data-dependent trip count, no division inside.
template <int N>
__device__ __forceinline__ double clenshaw(const double (&c)[N], double t) {
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = N - 1; j >= 1; --j) {
        const double b0 = fma(2.0 * t, b1, c[j] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(t, b1, c[0] - b2);
}

// F(x) for |x| < 1: C = x sum c_n x^4n, S = x^3 sum s_n x^4n (Horner).
__device__ __forceinline__ c64 fresnel_small(double x) {
    using namespace fresnel_data;
    const double x2 = x * x, t = x2 * x2;
    double c = kSeriesC[kSeriesTerms - 1], sn = kSeriesS[kSeriesTerms - 1];
#pragma unroll
    for (int n = kSeriesTerms - 2; n >= 0; --n) {
        c = fma(c, t, kSeriesC[n]);
        sn = fma(sn, t, kSeriesS[n]);
    }
    return {x * c, x * x2 * sn};
}

// G(x) = g(x) + i f(x) for x >= 1.  The expansion of each u interval is run
// under a wave-uniform test, so that its coefficients are read with uniform
// (scalar) loads; lanes outside the interval keep their values.
__device__ __forceinline__ c64 fresnel_aux(double x) {
    using namespace fresnel_data;
    const double u = 1.0 / (x * x);
    const int iv = u < kUHi[0] ? 0 : u < kUHi[1] ? 1 : u < kUHi[2] ? 2 : 3;
    double pf = 0.0, pg = 0.0;
    auto fit = [&](const auto &cf, const auto &cg, int i) {
        if (__any(iv == i) && iv == i) {
            const double t = (2.0 * u - (kUHi[i] + kULo[i])) / (kUHi[i] - kULo[i]);
            pf = clenshaw(cf, t);
            pg = clenshaw(cg, t);
        }
    };
    fit(kPhiF0, kPhiG0, 0);
    fit(kPhiF1, kPhiG1, 1);
    fit(kPhiF2, kPhiG2, 2);
    fit(kPhiF3, kPhiG3, 3);
    const double ipx = 1.0 / (kPiD * x);  // f = phi_f / (pi x), g = phi_g / (pi^2 x^3)
    return {pg * u * ipx * (1.0 / kPiD), pf * ipx};
}

// H(x) = F(x) exp(-i pi x^2 / 2); H(-x) = -H(x).
__device__ c64 fresnel_h(double x) {
    const double ax = fabs(x);
    const c64 rot = cis_pi(-0.5 * ax * ax);
    c64 h;
    if (ax < 1.0) {
        h = cmul(fresnel_small(ax), rot);
    } else {
        const c64 g = fresnel_aux(ax);
        h = {0.5 * (rot.re - rot.im) - g.re, 0.5 * (rot.re + rot.im) - g.im};  // (1 + i)/2 rot - G
    }
    return x < 0.0 ? c64{-h.re, -h.im} : h;
}

// A(q, z) = int_0^1 exp(2 pi i [(q - z/2) u + z u^2 / 2]) du: the Fourier
// response at offset q bins of a unit tone whose frequency drifts by z bins
// over the observation (Sec. 2); e2q = exp(2 pi i q) is passed in (it is the
// same for every integer shift of q).  z = 0: exp(i pi q) sin(pi q) / (pi q).
// z > 0: with p = q - z/2, Y = p sqrt(2/z), Z = Y + sqrt(2z) (so that
// pi (Z^2 - Y^2) / 2 = 2 pi q),
//   A = exp(-i pi Y^2 / 2) (F(Z) - F(Y)) / sqrt(2z) = (e2q H(Z) - H(Y)) / sqrt(2z);
// when |Y|, |Z| >= 1 on one side the (1 + i)/2 parts of H cancel exactly and
// A = (G(Y) - e2q G(Z)) / sqrt(2z) (both positive) or
// (e2q G(-Z) - G(-Y)) / sqrt(2z) (both negative).  z < 0: conj(A(-q, -z)).
__device__ c64 accel_response(double q, double z, c64 e2q) {
    if (z == 0.0) {
        if (q == rint(q)) return q == 0.0 ? c64{1.0, 0.0} : c64{0.0, 0.0};
        return cscale(cis_pi(q), sinpi(q) / (kPiD * q));
    }
    bool neg = false;
    if (z < 0.0) {
        neg = true;
        q = -q;
        z = -z;
        e2q.im = -e2q.im;
    }
    const double p = q - 0.5 * z;
    const double s = sqrt(2.0 / z);
    const double Y = p * s, Zv = (p + z) * s;
    const double pre = 1.0 / sqrt(2.0 * z);
    c64 a;
    if (Y >= 1.0) {
        a = csub(fresnel_aux(Y), cmul(e2q, fresnel_aux(Zv)));
    } else if (Zv <= -1.0) {
        a = csub(cmul(e2q, fresnel_aux(-Zv)), fresnel_aux(-Y));
    } else {
        a = csub(cmul(e2q, fresnel_h(Zv)), fresnel_h(Y));
    }
    a = cscale(a, pre);
    return neg ? c64{a.re, -a.im} : a;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Normalised spectrum value Xhat[k] = X[k] sqrt(ln2 / m(k)) (X itself when
// med is NULL), in FP64.
struct Spectrum {
    const float2 *X;
    const double *med;
    int W;
    int64_t nb, nblk;
    __device__ c64 at(int64_t k) const {
        const float2 x = X[k];
        const double f = med ? sqrt(kLn2 / median_curve(med, nblk, W, nb, k)) : 1.0;
        return {double(x.x) * f, double(x.y) * f};
    }
};

// P(r, z) by one wave: Y = sum_{k in K(r)} Xhat[k] conj(A(r - k, z)) over the
// bins within h of r, normalised by sum_{k in K(r)} |A(r - k, z)|^2; Xhat is
// zero outside [0, nb).  The result is valid in every lane.
// (r, z) must be finite and below 2^50 in magnitude (NaN otherwise), so
// that the 2h or 2h + 1 offsets r - k are exact.
__device__ double wave_power(const Spectrum &sp, int h, double r, double z, int lane) {
    if (!(fabs(r) < 0x1p50) || !(fabs(z) < 0x1p50)) return NAN;
    const double klo = ceil(r - double(h));
    const int ntap = int(floor(r + double(h)) - klo) + 1;  // 2h or 2h + 1
    double nre = 0.0, nim = 0.0, den = 0.0;
    const c64 e2q = cis_pi(2.0 * r);  // exp(2 pi i (r - k)) for every integer k
    for (int t = lane; t < ntap; t += 64) {
        const double kk = klo + double(t);
        const c64 a = accel_response(r - kk, z, e2q);
        den += cnorm2(a);
        const int64_t k = int64_t(kk);
        if (k >= 0 && k < sp.nb) {
            const c64 x = sp.at(k);
            nre += x.re * a.re + x.im * a.im;  // x conj(a)
            nim += x.im * a.re - x.re * a.im;
        }
    }
    nre = wave_sum(nre);
    nim = wave_sum(nim);
    den = wave_sum(den);
    return (nre * nre + nim * nim) / den;
}

// Point i (0..7) of a search level around (r, z): z-offset major, then
// r-offset, each in -1, 0, +1, the centre skipped.
__device__ __forceinline__ void level_point(int i, double r, double z, double sr, double sz, double &rr,
                                            double &zz) {
    const int g = i < 4 ? i : i + 1;
    const int b = g / 3 - 1, a = g % 3 - 1;
    rr = r + double(a) * sr;
    zz = z + double(b) * sz;
}

// The workgroup's harmonic sums S(r_i, z_i) = sum_{j=1}^{nh} P(j r_i, j z_i)
// for npts points (the level's neighbours, or the centre when npts is 1):
// waves take the (point, harmonic) pairs in turn, the per-pair powers meet in
// LDS (pw) and thread i sums point i's in the order j = 1 .. nh into S[i].
// On return S is visible to every thread.
__device__ void eval_points(const Spectrum &sp, int h, int nh, int npts, double r, double z, double sr, double sz,
                            double *pw, double *S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int pj = wave; pj < npts * nh; pj += nwaves) {
        const int i = pj / nh, j = pj - i * nh + 1;
        double rr = r, zz = z;
        if (npts > 1) level_point(i, r, z, sr, sz, rr, zz);
        const double p = wave_power(sp, h, double(j) * rr, double(j) * zz, lane);
        if (lane == 0) pw[pj] = p;
    }
    __syncthreads();
    if (int(threadIdx.x) < npts) {
        double s = 0.0;
        for (int j = 0; j < nh; ++j) s += pw[threadIdx.x * nh + j];
        S[threadIdx.x] = s;
    }
    __syncthreads();
}

// One workgroup per candidate (persistent grid): start at the fundamental
// r = k / (nh cpb), z = ((iz - izc) dz) / nh (cpb = 2 on a half-bin plane), then per level l = 1 .. levels move
// to the best of the 8 neighbours at steps (2^-l / nh, (dz 2^-l) / nh) when
// it is strictly larger than the centre (earlier points win ties); points
// whose top harmonic drifts beyond the bank (|nh z| > zmax) are skipped.
__global__ __launch_bounds__(RF_THREADS) void k_refine(Spectrum sp, int h, int izc, double dz, double zmax,
                                                       int cpb, int levels, const uint32_t *__restrict__ count,
                                                       uint32_t cap, fdas_cand *__restrict__ cands) {
    __shared__ double pw[RF_POINTS * RF_MAX_NH];
    __shared__ double S[RF_POINTS];
    const uint32_t n = min(*count, cap);
    for (uint32_t c = blockIdx.x; c < n; c += gridDim.x) {
        const int64_t k = cands[c].k;
        const int iz = cands[c].iz;
        const int nh = cands[c].nharm;
        if (nh < 1 || nh > RF_MAX_NH) continue;  // uniform over the workgroup
        double r = double(k) / (double(nh) * double(cpb));
        double z = (double(iz - izc) * dz) / double(nh);
        double best = 0.0;
        // level 0 evaluates the centre alone
        for (int l = 0; l <= levels; ++l) {
            const double sr = ldexp(1.0, -l) / double(nh);
            const double sz = (dz * ldexp(1.0, -l)) / double(nh);
            eval_points(sp, h, nh, l == 0 ? 1 : RF_POINTS, r, z, sr, sz, pw, S);
            if (l == 0) {
                best = S[0];
                continue;
            }
            double br = r, bz = z;
            for (int i = 0; i < RF_POINTS; ++i) {
                double rr, zz;
                level_point(i, r, z, sr, sz, rr, zz);
                if (fabs(double(nh) * zz) > zmax) continue;
                if (S[i] > best) {
                    best = S[i];
                    br = rr;
                    bz = zz;
                }
            }
            r = br;
            z = bz;
        }
        if (threadIdx.x == 0) {
            cands[c].r = r;
            cands[c].z = z;
            cands[c].power = float(best);
        }
    }
}

// Significance of the refined records' powers, one thread per record (kept
// out of k_refine, where its special functions would set the register budget
// of the whole search).
__global__ __launch_bounds__(256) void k_refine_sigma(const uint32_t *__restrict__ count, uint32_t cap,
                                                      fdas_cand *__restrict__ cands) {
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int nh = cands[i].nharm;
        if (nh < 1 || nh > RF_MAX_NH) continue;
        cands[i].sigma = float(significance_d(double(cands[i].power), nh));
    }
}

// S(r_i, z_i) for listed points, one workgroup per point (persistent grid).
__global__ __launch_bounds__(RF_POINT_THREADS) void k_interp_points(Spectrum sp, int h, const double *__restrict__ r,
                                                              const double *__restrict__ z,
                                                              const int32_t *__restrict__ nh, int64_t n,
                                                              double *__restrict__ out) {
    __shared__ double pw[RF_MAX_NH];
    __shared__ double S[1];
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int m = nh[i];
        if (m < 1 || m > RF_MAX_NH) {
            if (threadIdx.x == 0) out[i] = NAN;
            continue;
        }
        eval_points(sp, h, m, 1, r[i], z[i], 0.0, 0.0, pw, S);
        if (threadIdx.x == 0) out[i] = S[0];
    }
}

Spectrum make_spectrum(const float2 *X, const double *med, int W, int64_t nb) {
    Spectrum sp;
    sp.X = X;
    sp.med = med;
    sp.W = W;
    sp.nb = nb;
    sp.nblk = (nb + W - 1) / W;
    return sp;
}

}  // namespace

hipError_t launch_refine(const float2 *X, const double *med, int W, int64_t nb, int h, int izc, double dz,
                         double zmax, int cpb, int levels, const uint32_t *count, uint32_t cap, fdas_cand *cands,
                         int workgroups, hipStream_t st) {
    if (cap == 0 || levels <= 0) return hipSuccess;
    if (levels > 30 || workgroups <= 0 || nb <= 0 || W <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine, dim3(unsigned(workgroups)), dim3(RF_THREADS), 0, st,
                       make_spectrum(X, med, W, nb), h, izc, dz, zmax, cpb, levels, count, cap, cands);
    hipLaunchKernelGGL(k_refine_sigma, dim3(unsigned(workgroups)), dim3(256), 0, st, count, cap, cands);
    return hipGetLastError();
}

// Records and count of fdas_refine_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never hands the
// array's name to a kernel or a copy (on the host it is only a stand-in for
// the symbol); it uses the device address hipGetSymbolAddress returns for
// the current device, looked up once per device and kept.
constexpr size_t kRefineScratchBytes = size_t(FDAS_REFINE_NOALLOC_MAX) * sizeof(fdas_cand) + 256;
static __device__ __align__(256) unsigned char scratch[kRefineScratchBytes];

hipError_t refine_noalloc_scratch(void **out, size_t *bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    *bytes = kRefineScratchBytes;
    return hipSuccess;
}

hipError_t launch_interp_points(const float2 *X, const double *med, int W, int64_t nb, int h, const double *r,
                                const double *z, const int32_t *nh, int64_t n, double *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (nb <= 0 || W <= 0) return hipErrorInvalidValue;
    const int64_t grid = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(k_interp_points, dim3(unsigned(grid)), dim3(RF_POINT_THREADS), 0, st,
                       make_spectrum(X, med, W, nb), h, r, z, nh, n, out);
    return hipGetLastError();
}

}  // namespace fdas
