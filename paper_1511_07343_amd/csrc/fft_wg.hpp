// Workgroup-resident complex FFT for gfx950 (CDNA4, wave64).
//
// One workgroup of NT threads transforms S = 2^LOG2S complex float32 points.
// Each thread keeps R = S / NT points in registers; data enter and leave in
// the strided layout "thread t holds element t + NT*m in v[m]", which makes
// every global load and store of a transform coalesced across the wavefront.
//
// The transform is a Stockham autosort FFT (no bit-reversal pass): pass p of
// radix Rp = 2^bits(p) takes the Rp inputs x[j + r*S/Rp] of butterfly j,
// multiplies input r by the twiddle exp(DIR 2 pi i r (j mod Ns) / (Ns Rp)),
// runs an Rp-point DFT in registers and writes output r to position
// (j div Ns) Ns Rp + (j mod Ns) + r Ns, where Ns is the product of the earlier
// radices.  Between passes the points go through LDS (one exchange per pass
// boundary); the first pass reads registers and the last pass writes them.
// Each thread runs R / Rp butterflies per pass (j = t + NT*b).
//
// The register DFTs are recursive radix-2 decimation-in-time with compile-time
// twiddles; multiplications by 1, -1 and +-i are specialised away, and the
// other twiddles are folded into their butterfly (see bfly).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace fdas {

// ------------------------------------------------------------------ complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Products with their fused multiply-adds written out, so that the rounding
// of a result does not depend on how the compiler contracts the surrounding
// code (one multiply, then one fma, in this order).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float cnorm(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// ----------------------------------------------------- compile-time helpers
template <int I, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(std::forward<F>(f));
    }
}

constexpr double kPiD = 3.14159265358979323846264338327950288;

// sin / cos by Taylor series on |x| <= pi (compile-time constants only).
constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / double((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / double((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}

constexpr int ct_log2(int n) { return n <= 1 ? 0 : 1 + ct_log2(n / 2); }

// a * exp(DIR * 2 pi i K / N) with K, N compile-time.
template <int K, int N, int DIR>
__device__ __forceinline__ float2 rot(float2 a) {
    constexpr int k = ((K % N) + N) % N;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (2 * k == N) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (4 * k == N) {  // exp(DIR i pi/2) = DIR i
        return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    } else if constexpr (4 * k == 3 * N) {  // -DIR i
        return DIR > 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
    } else {
        // reduce the angle to (-pi, pi] for an accurate series
        constexpr double ang0 = 2.0 * kPiD * double(k) / double(N);
        constexpr double ang = ang0 > kPiD ? ang0 - 2.0 * kPiD : ang0;
        constexpr float c = float(ct_cos(ang));
        constexpr float s = float(DIR * ct_sin(ang));
        if constexpr (8 * k == N || 8 * k == 3 * N || 8 * k == 5 * N || 8 * k == 7 * N) {
            // |c| = |s| = 1/sqrt(2): two adds and two multiplies
            constexpr float m = c > 0 ? c : -c;
            if constexpr ((c > 0) == (s > 0)) {
                const float x = a.x - a.y, y = a.x + a.y;
                return c > 0 ? make_float2(m * x, m * y) : make_float2(-m * x, -m * y);
            } else {
                const float x = a.x + a.y, y = a.y - a.x;
                return c > 0 ? make_float2(m * x, m * y) : make_float2(-m * x, -m * y);
            }
        } else {
            return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
        }
    }
}

// Radix-2 butterfly with a compile-time twiddle w = exp(DIR 2 pi i K / N):
// lo = e + w o, hi = e - w o.  A twiddle that is not a multiple of i is
// factored as w = c (1 + i tan) (or s (cot + i) where |sin| > |cos|, so the
// ratio stays within [-1, 1]): the ratio's product is two fused
// multiply-adds and the scale folds into the four output fused
// multiply-adds, 6 instructions instead of the 8 of a product and two
// complex additions.
template <int K, int N, int DIR>
__device__ __forceinline__ void bfly(float2 e, float2 o, float2 &lo, float2 &hi) {
    constexpr int k = ((K % N) + N) % N;
    if constexpr (k == 0 || 2 * k == N || 4 * k == N || 4 * k == 3 * N) {
        const float2 t = rot<K, N, DIR>(o);
        lo = cadd(e, t);
        hi = csub(e, t);
    } else {
        constexpr double ang0 = 2.0 * kPiD * double(k) / double(N);
        constexpr double ang = ang0 > kPiD ? ang0 - 2.0 * kPiD : ang0;
        constexpr double c = ct_cos(ang);
        constexpr double sn = DIR * ct_sin(ang);
        constexpr bool by_cos = (c < 0 ? -c : c) >= (sn < 0 ? -sn : sn);
        float2 w;
        float f;
        if constexpr (by_cos) {
            // w o = c (o.x - o.y t, o.y + o.x t), t = s / c
            constexpr float t = float(sn / c);
            w = make_float2(fmaf(-o.y, t, o.x), fmaf(o.x, t, o.y));
            f = float(c);
        } else {
            // w o = s (o.x q - o.y, o.y q + o.x), q = c / s
            constexpr float q = float(c / sn);
            w = make_float2(fmaf(o.x, q, -o.y), fmaf(o.y, q, o.x));
            f = float(sn);
        }
        lo = make_float2(fmaf(f, w.x, e.x), fmaf(f, w.y, e.y));
        hi = make_float2(fmaf(-f, w.x, e.x), fmaf(-f, w.y, e.y));
    }
}

// In-register DFT of N points (natural order in and out), direction DIR.
template <int N, int DIR>
__device__ __forceinline__ void dft_reg(float2 (&u)[N]) {
    if constexpr (N == 2) {
        const float2 a = u[0], b = u[1];
        u[0] = cadd(a, b);
        u[1] = csub(a, b);
    } else if constexpr (N > 2) {
        float2 e[N / 2], o[N / 2];
#pragma unroll
        for (int m = 0; m < N / 2; ++m) {
            e[m] = u[2 * m];
            o[m] = u[2 * m + 1];
        }
        dft_reg<N / 2, DIR>(e);
        dft_reg<N / 2, DIR>(o);
        static_for<0, N / 2>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            bfly<k, N, DIR>(e[k], o[k], u[k], u[k + N / 2]);
        });
    }
}

// ---------------------------------------------------------------- geometry
template <int LOG2S_, int NT_>
struct FftShape {
    static constexpr int LOG2S = LOG2S_;
    static constexpr int NT = NT_;
    static constexpr int S = 1 << LOG2S;
    static constexpr int LOG2NT = ct_log2(NT);
    static_assert((1 << LOG2NT) == NT, "NT must be a power of two");
    static constexpr int LOG2R = LOG2S - LOG2NT;
    static_assert(LOG2R >= 1 && LOG2R <= 5, "2..32 points per thread");
    static constexpr int R = 1 << LOG2R;
    static constexpr int NPASS = (LOG2S + LOG2R - 1) / LOG2R;
    static constexpr int bits(int p) { return LOG2S / NPASS + (p < LOG2S % NPASS ? 1 : 0); }
    static constexpr int radix(int p) { return 1 << bits(p); }
    static constexpr int ns(int p) { return p == 0 ? 1 : ns(p - 1) * radix(p - 1); }
    static constexpr int nbf(int p) { return R / radix(p); }
    // LDS padding: one float2 every 32 keeps the strided writes of the early
    // passes off a single bank.
    static constexpr int pad(int i) { return i + (i >> 5); }
    static constexpr int LDS_FLOAT2 = S + (S >> 5);
    // Twiddles of pass p > 0 are stored for butterfly b = 0 only: with NT and
    // Ns powers of two, (t + NT b) mod Ns = (t mod Ns) + (NT b mod Ns), so the
    // twiddle of butterfly b is the stored one times the compile-time rotation
    // exp(DIR 2 pi i r (NT b mod Ns) / (Ns Rp)).
    static constexpr int ntw(int p) { return p == 0 ? 0 : radix(p) - 1; }
    static constexpr int tw_off(int p) { return p == 0 ? 0 : tw_off(p - 1) + ntw(p - 1); }
    static constexpr int NTW = tw_off(NPASS);
};
__device__ __forceinline__ int pad_idx(int i) { return i + (i >> 5); }
// pad_idx(base + r Ns) for the Rp outputs of a butterfly whose first one is
// base: with Ns a multiple of 32, or the butterfly's Ns Rp elements inside one
// aligned run of 32 (base mod Ns Rp < Ns), the padding grows linearly in r,
// so the address is pad_idx(base) plus a compile-time multiple of r: an
// immediate offset, where the compiler would otherwise keep every output's
// address in a register of its own across the caller's loops.
template <int Ns, int Rp>
__device__ __forceinline__ int pad_slot(int pb, int base, int r) {
    if constexpr (Ns % 32 == 0) return pb + r * (Ns + Ns / 32);
    else if constexpr (32 % (Ns * Rp) == 0) return pb + r * Ns;
    else return pad_idx(base + r * Ns);
}
// pad_idx(t + NT m) with NT a multiple of 32
template <int NT>
__device__ __forceinline__ int pad_strided(int pt, int m) {
    static_assert(NT % 32 == 0, "threads a multiple of 32");
    return pt + m * (NT + NT / 32);
}

// Per-thread twiddles of every pass, computed once and reused for every
// transform the thread takes part in.  Twiddle r of a pass is w^r with
// w = exp(DIR 2 pi i jj / (Ns Rp)): the powers r = 2^b come from sincospif
// of an exact binary fraction, every other r is one product, w^(r - 2^b)
// times w^(2^b) for the highest bit b of r (at most log2(Rp) - 1 roundings
// deep), which replaces Rp - 1 - log2(Rp) sincospif evaluations per pass.
template <class Sh, int DIR>
struct Twiddles {
    float2 w[Sh::NTW > 0 ? Sh::NTW : 1];

    __device__ __forceinline__ void init(int t) {
        static_for<1, Sh::NPASS>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int Rp = Sh::radix(p);
            constexpr int Ns = Sh::ns(p);
            constexpr int o = Sh::tw_off(p) - 1;  // w^r at w[o + r]
            const int jj = t & (Ns - 1);
            static_for<1, Rp>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                constexpr int hb = 1 << ct_log2(r);  // highest power of two <= r
                if constexpr (hb == r) {
                    // angle = DIR 2 pi r jj / (Ns Rp); the sincospi argument is exact
                    const float arg = float(DIR * 2 * r * jj) / float(Ns * Rp);
                    float sn, c;
                    sincospif(arg, &sn, &c);
                    w[o + r] = make_float2(c, sn);
                } else {
                    w[o + r] = cmul(w[o + (r - hb)], w[o + hb]);
                }
            });
        });
    }
};

// The transform.  v: registers in strided layout (see top); lds: workgroup
// buffer of Sh::LDS_FLOAT2 float2 (SPLIT: of Sh::LDS_FLOAT2 floats).  The
// caller must not touch lds between the call's first write and its return.
// On return every thread has passed a barrier after its last LDS read, so lds
// may be reused at once.
// SPLIT: a pass keeps its outputs in registers and exchanges the real parts,
// then the imaginary parts, through half the LDS (two more barriers per
// exchange); the values and so the results are those of the one-round form.
template <class Sh, int DIR, bool SPLIT = false>
__device__ __forceinline__ void fft_wg(float2 (&v)[Sh::R], float2 *lds, const Twiddles<Sh, DIR> &tw,
                                       int t) {
    static_for<0, Sh::NPASS>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int Rp = Sh::radix(p);
        constexpr int Ns = Sh::ns(p);
        constexpr int nb = Sh::nbf(p);
        constexpr bool last = (p == Sh::NPASS - 1);
        static_for<0, nb>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            float2 u[Rp];
#pragma unroll
            for (int r = 0; r < Rp; ++r) u[r] = v[b + r * nb];
            if constexpr (p > 0) {
                constexpr int off = (Sh::NT * b) & (Ns - 1);
                static_for<1, Rp>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    u[r] = rot<r * off, Ns * Rp, DIR>(cmul(u[r], tw.w[Sh::tw_off(p) + (r - 1)]));
                });
            }
            dft_reg<Rp, DIR>(u);
            if constexpr (last || SPLIT) {
                // (SPLIT: output r of butterfly b waits in its input's register)
#pragma unroll
                for (int r = 0; r < Rp; ++r) v[b + r * nb] = u[r];
            } else {
                const int j = t + Sh::NT * b;
                const int base = (j / Ns) * Ns * Rp + (j & (Ns - 1));
                const int pb = pad_idx(base);
#pragma unroll
                for (int r = 0; r < Rp; ++r) lds[pad_slot<Ns, Rp>(pb, base, r)] = u[r];
            }
        });
        if constexpr (!last && !SPLIT) {
            __syncthreads();
            const int pt = pad_idx(t);
#pragma unroll
            for (int m = 0; m < Sh::R; ++m) v[m] = lds[pad_strided<Sh::NT>(pt, m)];
            __syncthreads();
        } else if constexpr (!last) {
            float *__restrict__ lf = reinterpret_cast<float *>(lds);
            static_for<0, 2>([&](auto hc) {
                constexpr int half = decltype(hc)::value;
                static_for<0, nb>([&](auto bc) {
                    constexpr int b = decltype(bc)::value;
                    const int j = t + Sh::NT * b;
                    const int base = (j / Ns) * Ns * Rp + (j & (Ns - 1));
                    const int pb = pad_idx(base);
#pragma unroll
                    for (int r = 0; r < Rp; ++r)
                        lf[pad_slot<Ns, Rp>(pb, base, r)] = half ? v[b + r * nb].y : v[b + r * nb].x;
                });
                __syncthreads();
                const int pt = pad_idx(t);
#pragma unroll
                for (int m = 0; m < Sh::R; ++m) {
                    const float q = lf[pad_strided<Sh::NT>(pt, m)];
                    if constexpr (half) v[m].y = q; else v[m].x = q;
                }
                __syncthreads();
            });
        }
    });
}

}  // namespace fdas
