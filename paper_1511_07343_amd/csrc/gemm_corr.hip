// Precision variant of the correlation: Eq. (1) of Sec. 2 evaluated directly,
// as one real matrix product on the MFMA units with BF16 or FP16 operands and
// FP32 accumulation, instead of the overlap-save FFT path.
//
// Y_z[k] = sum_{q=-h..h} Xhat[k - q] T_z[q] is, with q' = q + h and the real
// and imaginary parts interleaved along K (c = 2 q' + part),
//   [Y_re | Y_im] = A B,  A[k][c] = (Re, Im) Xhat[k - q' + h],
//   B = [[ Re T, Im T], [-Im T, Re T]]   (rows: Re / Im of the input,
//                                          columns: Re / Im of the output).
// A is a Toeplitz matrix: row k + 1 is row k shifted by one complex value, so
// a block of rows needs only a window of the spectrum.  The power |Y|^2 and
// its screening code go to the same plane layout the FFT path writes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "kernels.hpp"

namespace fdas {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// v_mfma_f32_16x16x32_{bf16,f16}: lane l holds A[l % 16][8 (l / 16) + s] and
// B[8 (l / 16) + s][l % 16] (s < 8) and receives D[4 (l / 16) + r][l % 16]
// (r < 4).
template <bool BF16>
struct Mfma;
template <>
struct Mfma<true> {
    static __device__ __forceinline__ f32x4 op(uint4 a, uint4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    }
};
template <>
struct Mfma<false> {
    static __device__ __forceinline__ f32x4 op(uint4 a, uint4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    }
};

// 16-bit encodings, round to nearest even (the same conversions on host and
// device).
template <bool BF16>
__host__ __device__ inline uint16_t to_half_bits(float x) {
    if constexpr (BF16) return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
    else return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
}

constexpr int GM_WAVES = 4;
constexpr int GM_RT = 8;                         // row tiles of 16 bins per wave
constexpr int GM_ROWS = GM_WAVES * GM_RT * 16;   // bins per row block
constexpr int GM_TZ = 16;                        // templates per slice
constexpr int GM_CT = 2 * GM_TZ / 16;            // column tiles: Re, then Im, of the slice's templates
constexpr int GM_WIN = 16;                       // A fragments kept per wave (power of two >= GM_RT + 1)
constexpr int GM_FRAG = 64;                      // 16-byte fragments per MFMA operand (one per lane)
constexpr int GM_SLICE_FRAGS = GM_CT * GM_FRAG;  // B fragments of one K step of a slice
constexpr int GM_WORDS(int nk) { return GM_ROWS + 16 * nk; }  // window words per copy
// Words from one copy of the window to the next: at least GM_WORDS(nk), and
// 16 more than a multiple of 64, so that the four lanes of a fragment read
// that take the four copies start 16 banks apart (with a stride that is a
// multiple of 64 words they start on the same bank: a 4-way conflict on every
// A-fragment read).
constexpr int GM_STRIDE(int nk) { return GM_WORDS(nk) + ((16 - GM_WORDS(nk)) % 64 + 64) % 64; }
// window words loaded per thread (copies are written from registers)
constexpr int GM_WLOAD = (GM_WORDS(GM_MAX_KSTEPS) + 3 + 64 * GM_WAVES - 1) / (64 * GM_WAVES);

// Templates scaled by 16 (exactly) so that FP16 keeps the tails of the taps
// away from its subnormal range; powers are scaled back by 1/256.
constexpr double GM_TAP_SCALE = 16.0;

// Word k = (Re, Im) of Xhat[k] as two 16-bit floats, Re in the low half.
template <bool BF16>
__global__ __launch_bounds__(256) void k_lowp_spectrum(const float2 *__restrict__ X, const double *__restrict__ med,
                                                       int W, int64_t nb, uint32_t *__restrict__ out) {
    const int64_t g = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (g >= nb) return;
    float2 x = X[g];
    if (med) {
        const int64_t nblk = (nb + W - 1) / W;
        const double mk = median_curve(med, nblk, W, nb, g);
        const float sc = mk > 0.0 ? float(sqrt(kLn2 / mk)) : 0.f;
        x = make_float2(x.x * sc, x.y * sc);
    }
    out[g] = uint32_t(to_half_bits<BF16>(x.x)) | (uint32_t(to_half_bits<BF16>(x.y)) << 16);
}

// One workgroup: the B fragments of one template slice (all K) staged in LDS,
// then row blocks of GM_ROWS bins, each through a spectrum window in LDS.
// The LDS holds gemm_lds_bytes(nk): slices of 16 templates keep it small
// enough for two workgroups per CU up to about 30 K steps, so that the MFMA
// units of a SIMD have two waves to switch between.
// Wave w owns rows [128 w, 128 w + 128) of a block (8 row tiles) and all
// GM_CT column tiles (Re of the slice's templates, 16 per tile, then Im).
//
// The A fragment of (row tile rt, K step ks) holds window words
// u = (GM_ROWS - 1 - row) + 16 ks + 4 (l / 16) .. + 3, which depend on ks - rt
// only: F(d) with d = ks - rt.  A wave keeps F(ks - 15) .. F(ks + 1) in
// registers and loads one new fragment per K step.  The window is stored in
// four copies shifted by one word, so that every lane's fragment is a 16-byte
// aligned LDS read (copy (3 - l % 16) mod 4).
//
// The next block's window is loaded into registers before this block's
// powers are stored, so that the stores drain while the next block runs
// (vector-memory counters count loads and stores together).
template <bool BF16>
__global__ __launch_bounds__(64 * GM_WAVES, 2) void k_corr_gemm(
    const uint32_t *__restrict__ xl, int64_t nb, int h, int nk, const uint4 *__restrict__ bfrag, int nz, int nsl,
    int64_t nrb, int64_t per, float power_scale, float *__restrict__ plane, uint8_t *__restrict__ codes,
    float code_inv) {
    extern __shared__ uint4 gm_lds[];
    uint4 *__restrict__ bl = gm_lds;  // nk GM_SLICE_FRAGS fragments
    // then 4 copies of GM_WORDS(nk) words, GM_STRIDE(nk) words apart
    uint32_t *__restrict__ win = reinterpret_cast<uint32_t *>(gm_lds + nk * GM_SLICE_FRAGS);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int i16 = lane & 15, kg = lane >> 4;
    const int uw = GM_WORDS(nk);
    const int ust = GM_STRIDE(nk);
    const int sig = (3 - i16) & 3;
    // word of F(0) in copy sig (a multiple of 4; F(d) is 16 d words further)
    const int fbase = sig * ust + (GM_ROWS - 1 - 128 * wave - i16) + 4 * kg - sig;

    // this workgroup's items: (slice, row block) pairs [item0, item1), slice-major
    const int64_t total = int64_t(nsl) * nrb;
    const int64_t item0 = int64_t(blockIdx.x) * per;
    const int64_t item1 = min(total, item0 + per);
    if (item0 >= item1) return;
    // window words W[u] = xl[P0 - u], u < uw + 3 (zero outside the spectrum),
    // thread t holding u = t + 256 i
    uint32_t wreg[GM_WLOAD];
    auto load_window = [&](int64_t item) {
        const int sl = int(item / nrb);
        const int64_t p0 = (item - int64_t(sl) * nrb) * GM_ROWS + GM_ROWS - 1 + h;
#pragma unroll
        for (int i = 0; i < GM_WLOAD; ++i) {
            const int u = t + 64 * GM_WAVES * i;
            const int64_t p = p0 - u;
            wreg[i] = (u < uw + 3 && p >= 0 && p < nb) ? xl[p] : 0u;
        }
    };
    load_window(item0);
    int cur_slice = -1;
    for (int64_t item = item0; item < item1; ++item) {
        const int sl = int(item / nrb);
        const int64_t k0 = (item - int64_t(sl) * nrb) * GM_ROWS;
        __syncthreads();  // the previous item's LDS reads are done
        if (sl != cur_slice) {
            const uint4 *__restrict__ src = bfrag + int64_t(sl) * nk * GM_SLICE_FRAGS;
            for (int i = t; i < nk * GM_SLICE_FRAGS; i += 64 * GM_WAVES) bl[i] = src[i];
            cur_slice = sl;
        }
        // copy s holds W[v + s] at v
#pragma unroll
        for (int i = 0; i < GM_WLOAD; ++i) {
            const int u = t + 64 * GM_WAVES * i;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int v = u - c;
                if (v >= 0 && v < uw) win[c * ust + v] = wreg[i];
            }
        }
        __syncthreads();

        f32x4 acc[GM_RT][GM_CT];
#pragma unroll
        for (int rt = 0; rt < GM_RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < GM_CT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
        uint4 F[GM_WIN];
#pragma unroll
        for (int d = 1; d < GM_RT; ++d)  // F(-7) .. F(-1)
            F[(GM_WIN - d) % GM_WIN] = *reinterpret_cast<const uint4 *>(win + fbase - 16 * d);
        F[0] = *reinterpret_cast<const uint4 *>(win + fbase);
        uint4 b[GM_CT];
#pragma unroll
        for (int ct = 0; ct < GM_CT; ++ct) b[ct] = bl[ct * GM_FRAG + lane];
        for (int kb = 0; kb < nk; kb += GM_WIN) {
#pragma unroll
            for (int j = 0; j < GM_WIN; ++j) {
                const int ks = kb + j;
                if (ks < nk) {
                    // prefetch step ks + 1 (F(ks + 1) replaces F(ks - 15), no longer used)
                    uint4 bn[GM_CT];
                    if (ks + 1 < nk) {
                        F[(j + 1) % GM_WIN] = *reinterpret_cast<const uint4 *>(win + fbase + 16 * (ks + 1));
#pragma unroll
                        for (int ct = 0; ct < GM_CT; ++ct) bn[ct] = bl[((ks + 1) * GM_CT + ct) * GM_FRAG + lane];
                    }
#pragma unroll
                    for (int rt = 0; rt < GM_RT; ++rt) {
                        const uint4 a = F[(j - rt + GM_WIN) % GM_WIN];
#pragma unroll
                        for (int ct = 0; ct < GM_CT; ++ct) acc[rt][ct] = Mfma<BF16>::op(a, b[ct], acc[rt][ct]);
                    }
                    if (ks + 1 < nk) {
#pragma unroll
                        for (int ct = 0; ct < GM_CT; ++ct) b[ct] = bn[ct];
                    }
                }
            }
        }
        if (item + 1 < item1) load_window(item + 1);

        // powers: column tile c < GM_CT / 2 is Re of templates 16 c + i16, tile
        // c + GM_CT / 2 their Im; rows 4 (l / 16) + r of each row tile
#pragma unroll
        for (int half = 0; half < GM_CT / 2; ++half) {
            const int z = sl * GM_TZ + 16 * half + i16;
            if (z >= nz) continue;
            float *__restrict__ prow = plane + int64_t(z) * nb;
            uint8_t *__restrict__ qrow = codes + int64_t(z) * (nb / 2);
#pragma unroll
            for (int rt = 0; rt < GM_RT; ++rt) {
                const int64_t k = k0 + 128 * wave + 16 * rt + 4 * kg;
                if (k >= nb) continue;
                const f32x4 re = acc[rt][half], im = acc[rt][half + GM_CT / 2];
                float4 pw;
                pw.x = fmaf(re[0], re[0], im[0] * im[0]) * power_scale;
                pw.y = fmaf(re[1], re[1], im[1] * im[1]) * power_scale;
                pw.z = fmaf(re[2], re[2], im[2] * im[2]) * power_scale;
                pw.w = fmaf(re[3], re[3], im[3] * im[3]) * power_scale;
                *reinterpret_cast<float4 *>(prow + k) = pw;
                *reinterpret_cast<uint16_t *>(qrow + (k >> 1)) = block_codes4(pw, code_inv);
            }
        }
    }
}

}  // namespace

int gemm_ksteps(int h) { return (2 * (2 * h + 1) + 31) / 32; }

static size_t gemm_lds_bytes(int nk) { return size_t(nk * GM_SLICE_FRAGS + GM_STRIDE(nk)) * 16; }

size_t gemm_bank_bytes(int nz, int h) {
    return size_t((nz + GM_TZ - 1) / GM_TZ) * size_t(gemm_ksteps(h)) * GM_SLICE_FRAGS * 16;
}

void build_gemm_bank(const double *taps, int nz, int h, bool bf16, void *out) {
    const int ntap = 2 * h + 1, nk = gemm_ksteps(h), nsl = (nz + GM_TZ - 1) / GM_TZ;
    uint16_t *o = static_cast<uint16_t *>(out);
    size_t idx = 0;
    for (int sl = 0; sl < nsl; ++sl)
        for (int ks = 0; ks < nk; ++ks)
            for (int ct = 0; ct < GM_CT; ++ct)
                for (int l = 0; l < 64; ++l)
                    for (int s = 0; s < 8; ++s, ++idx) {
                        const int c = 32 * ks + 8 * (l / 16) + s;  // K index
                        const int col = 16 * ct + (l % 16);        // output column of the slice
                        const int qp = c / 2, part_in = c % 2;
                        const int z = sl * GM_TZ + (col % GM_TZ), part_out = col / GM_TZ;
                        double v = 0.0;
                        if (qp < ntap && z < nz) {
                            const double tr = taps[2 * (size_t(z) * ntap + qp)];
                            const double ti = taps[2 * (size_t(z) * ntap + qp) + 1];
                            v = part_in == 0 ? (part_out == 0 ? tr : ti) : (part_out == 0 ? -ti : tr);
                        }
                        const float f = float(v * GM_TAP_SCALE);
                        o[idx] = bf16 ? to_half_bits<true>(f) : to_half_bits<false>(f);
                    }
}

hipError_t launch_lowp_spectrum(const float2 *X, const double *med, int W, int64_t nb, bool bf16, uint32_t *out,
                                hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    const dim3 grid(unsigned((nb + 255) / 256));
    if (bf16) hipLaunchKernelGGL(k_lowp_spectrum<true>, grid, dim3(256), 0, st, X, med, W, nb, out);
    else hipLaunchKernelGGL(k_lowp_spectrum<false>, grid, dim3(256), 0, st, X, med, W, nb, out);
    return hipGetLastError();
}

hipError_t launch_corr_gemm(const uint32_t *xl, int64_t nb, int h, const void *bank, int nz, bool bf16,
                            int workgroups, float *plane, uint8_t *codes, float code_inv, hipStream_t st) {
    const int nk = gemm_ksteps(h);
    if (nk > GM_MAX_KSTEPS || nb % 4 != 0 || workgroups <= 0) return hipErrorInvalidValue;
    const int nsl = (nz + GM_TZ - 1) / GM_TZ;
    const int64_t nrb = (nb + GM_ROWS - 1) / GM_ROWS;
    const size_t lds = gemm_lds_bytes(nk);
    // workgroups per CU that fit beside each other (the LDS decides)
    int per_cu = 0;
    hipError_t e = bf16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_corr_gemm<true>, 64 * GM_WAVES, lds)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_corr_gemm<false>, 64 * GM_WAVES, lds);
    if (e != hipSuccess) return e;
    workgroups *= std::max(per_cu, 1);
    const int64_t per = (int64_t(nsl) * nrb + workgroups - 1) / workgroups;
    const int64_t grid = (int64_t(nsl) * nrb + per - 1) / per;
    const float scale = float(1.0 / (GM_TAP_SCALE * GM_TAP_SCALE));
    const uint4 *bf = static_cast<const uint4 *>(bank);
    if (bf16)
        hipLaunchKernelGGL(k_corr_gemm<true>, dim3(unsigned(grid)), dim3(64 * GM_WAVES), lds, st, xl, nb, h, nk, bf, nz,
                           nsl, nrb, per, scale, plane, codes, code_inv);
    else
        hipLaunchKernelGGL(k_corr_gemm<false>, dim3(unsigned(grid)), dim3(64 * GM_WAVES), lds, st, xl, nb, h, nk, bf,
                           nz, nsl, nrb, per, scale, plane, codes, code_inv);
    return hipGetLastError();
}

}  // namespace fdas
