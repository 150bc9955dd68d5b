// Candidate finishing on the device: order the harmonic-sum kernel's
// (unordered) records by (nharm, k, iz) with an LSD radix sort (per 8-bit
// digit a count kernel and a scatter kernel that scans the counts itself),
// then write the public records with r, z and the FP64 single-trial
// significance.
// The record count stays on the device: every kernel reads it and clamps it
// to the buffer capacity, so nothing waits for the host in between.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fdas.h"
#include "device_common.hpp"
#include "kernels.hpp"

namespace fdas {

namespace {

constexpr int RS_BLOCKS = 128;   // workgroups of the histogram and scatter passes
constexpr int RS_THREADS = 256;  // four waves
constexpr int RS_DIGITS = 256;   // 8-bit digits
constexpr int RS_AHEAD = 8;      // tiles of 256 records a scatter or count workgroup loads at once

__device__ __forceinline__ uint32_t clamp_count(const uint32_t *count, uint32_t cap) {
    const uint32_t c = *count;
    return c < cap ? c : cap;
}

__device__ __forceinline__ void block_range(uint32_t n, uint32_t &beg, uint32_t &end) {
    const uint32_t chunk = (n + RS_BLOCKS - 1) / RS_BLOCKS;
    beg = min(n, blockIdx.x * chunk);
    end = min(n, beg + chunk);
}

// Digit counts of a radix pass, block-major: hist[block * RS_DIGITS + digit]
// counts the records of `block`'s range (block_range) with that digit.

// key = (level nb + k) nz + iz, level = log2(nharm) in 0..4, k < nb, iz < nz:
// ascending keys are ascending (nharm, k, iz), and all keys are below
// 5 nb nz (32 bits, four 8-bit passes, at 2^23 samples and 201 templates).
// One workgroup per block range (RS_BLOCKS of them): the keys and values of
// the range and the first pass's digit counts of the range.
__global__ __launch_bounds__(RS_THREADS) void k_cand_keys(const DevCand *__restrict__ dc, const uint32_t *__restrict__ count,
                                                          uint32_t cap, int64_t nb, int nz, uint64_t *__restrict__ keys,
                                                          uint32_t *__restrict__ vals, uint32_t *__restrict__ hist) {
    __shared__ uint32_t lh[RS_DIGITS];
    const uint32_t n = clamp_count(count, cap);
    const int t = threadIdx.x;
    lh[t] = 0u;
    __syncthreads();
    uint32_t beg, end;
    block_range(n, beg, end);
    for (uint32_t i = beg + t; i < end; i += RS_THREADS) {
        const DevCand c = dc[i];
        const uint64_t level = uint64_t(31 - __clz(c.nharm));
        const uint64_t key = (level * uint64_t(nb) + uint64_t(uint32_t(c.k))) * uint64_t(nz) + uint64_t(uint32_t(c.iz));
        keys[i] = key;
        vals[i] = i;
        atomicAdd(&lh[uint32_t(key) & (RS_DIGITS - 1u)], 1u);
    }
    __syncthreads();
    hist[blockIdx.x * RS_DIGITS + t] = lh[t];
}

// Lists of at most SMALL records are sorted by one workgroup in LDS
// (bitonic, not stable, which is harmless: no two records share a key); the
// radix passes skip them.
constexpr uint32_t SMALL = 2048;
constexpr int SMALL_THREADS = 1024;

__global__ __launch_bounds__(SMALL_THREADS) void k_small_sort(const uint64_t *__restrict__ kin,
                                                              const uint32_t *__restrict__ vin,
                                                              const uint32_t *__restrict__ count, uint32_t cap,
                                                              uint32_t *__restrict__ vout) {
    __shared__ uint64_t key[SMALL];
    __shared__ uint32_t val[SMALL];
    const uint32_t n = clamp_count(count, cap);
    if (n > SMALL) return;
    const int t = threadIdx.x;
    for (uint32_t i = t; i < SMALL; i += SMALL_THREADS) {
        key[i] = i < n ? kin[i] : ~uint64_t(0);
        val[i] = i < n ? vin[i] : 0u;
    }
    for (uint32_t size = 2; size <= SMALL; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (uint32_t i = t; i < SMALL / 2; i += SMALL_THREADS) {
                const uint32_t lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t a = key[lo], b = key[hi];
                if ((a > b) == asc) {
                    key[lo] = b;
                    key[hi] = a;
                    const uint32_t v = val[lo];
                    val[lo] = val[hi];
                    val[hi] = v;
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = t; i < n; i += SMALL_THREADS) vout[i] = val[i];
}

// Digit counts of the pass at `shift` (passes after the first).
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ count, uint32_t cap, int shift,
                                                        uint32_t *__restrict__ hist) {
    __shared__ uint32_t lh[RS_DIGITS];
    const uint32_t n = clamp_count(count, cap);
    if (n <= SMALL) return;
    const int t = threadIdx.x;
    lh[t] = 0u;
    __syncthreads();
    uint32_t beg, end;
    block_range(n, beg, end);
    for (uint32_t batch = beg; batch < end; batch += RS_AHEAD * RS_THREADS) {
        uint64_t kk[RS_AHEAD];
#pragma unroll
        for (int q = 0; q < RS_AHEAD; ++q) {
            const uint32_t i = batch + uint32_t(q) * RS_THREADS + t;
            kk[q] = i < end ? keys[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < RS_AHEAD; ++q)
            if (batch + uint32_t(q) * RS_THREADS + t < end)
                atomicAdd(&lh[uint32_t(kk[q] >> shift) & (RS_DIGITS - 1u)], 1u);
    }
    __syncthreads();
    hist[blockIdx.x * RS_DIGITS + t] = lh[t];
}

// One pass of the LSD radix sort: a stable scatter of one 8-bit digit.
// Each workgroup first derives its output offsets from the pass's digit
// counts (digit t's total over all blocks and over the blocks before this
// one, then a scan of the totals over the digits); then it re-walks its range
// in tiles of 256 (one element per thread, element order = wave-major lane
// order): a lane's rank among same-digit lanes of its wave comes from 8
// ballots, wave offsets from LDS counts, and a running per-digit offset
// carries across tiles.
__global__ __launch_bounds__(RS_THREADS) void k_rs_pass(const uint64_t *__restrict__ kin,
                                                        const uint32_t *__restrict__ vin,
                                                        const uint32_t *__restrict__ count, uint32_t cap, int shift,
                                                        const uint32_t *__restrict__ hist, uint64_t *__restrict__ kout,
                                                        uint32_t *__restrict__ vout) {
    __shared__ uint32_t base[RS_DIGITS];
    __shared__ uint32_t cnt[RS_THREADS / 64][RS_DIGITS];
    __shared__ uint32_t wsum[RS_THREADS / 64];
    const uint32_t n = clamp_count(count, cap);
    if (n <= SMALL) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t before = 0, total = 0;
#pragma unroll 16
    for (int b = 0; b < RS_BLOCKS; ++b) {
        const uint32_t c = hist[b * RS_DIGITS + t];
        total += c;
        before += b < int(blockIdx.x) ? c : 0u;
    }
    uint32_t incl = total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t off = incl - total + before;
    for (int ww = 0; ww < w; ++ww) off += wsum[ww];
    base[t] = off;  // ordered before its first use by the tile loop's barrier
    uint32_t beg, end;
    block_range(n, beg, end);
    const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
    // RS_AHEAD tiles' keys and values are loaded together, so that the
    // tiles of a batch wait for memory once
    for (uint32_t batch = beg; batch < end; batch += RS_AHEAD * RS_THREADS) {
        uint64_t kk[RS_AHEAD];
        uint32_t vv[RS_AHEAD];
#pragma unroll
        for (int q = 0; q < RS_AHEAD; ++q) {
            const uint32_t i = batch + uint32_t(q) * RS_THREADS + t;
            kk[q] = i < end ? kin[i] : 0;
            vv[q] = i < end ? vin[i] : 0u;
        }
#pragma unroll
        for (int q = 0; q < RS_AHEAD; ++q) {
            const uint32_t tile = batch + uint32_t(q) * RS_THREADS;
            if (tile >= end) break;  // the same for every thread
#pragma unroll
            for (int ww = 0; ww < RS_THREADS / 64; ++ww) cnt[ww][t] = 0;
            __syncthreads();
            const uint32_t i = tile + t;
            const bool valid = i < end;
            const uint64_t key = kk[q];
            const uint32_t val = vv[q];
            const uint32_t d = valid ? uint32_t(key >> shift) & 255u : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(valid && bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t rank = __popcll(peers & lt_mask);
            if (valid && rank == 0) cnt[w][d] = __popcll(peers);
            __syncthreads();
            // thread t owns digit t: offsets of each wave within the tile
            uint32_t o = 0;
#pragma unroll
            for (int ww = 0; ww < RS_THREADS / 64; ++ww) {
                const uint32_t c = cnt[ww][t];
                cnt[ww][t] = o;
                o += c;
            }
            __syncthreads();
            if (valid) {
                const uint32_t pos = base[d] + cnt[w][d] + rank;
                kout[pos] = key;
                vout[pos] = val;
            }
            __syncthreads();
            base[t] += o;
        }
    }
}

// The public records of the first min(count, cap, out_cap) sorted records;
// with count_dst, also the six counter words there (out and count_dst may be
// device aliases of page-locked host memory).
__global__ __launch_bounds__(256) void k_cand_finalize(const DevCand *__restrict__ dc,
                                                       const uint32_t *__restrict__ order,
                                                       const uint32_t *__restrict__ count, uint32_t cap, int cpb,
                                                       double zmax, double dz, fdas_cand *__restrict__ out,
                                                       uint32_t out_cap, uint32_t *__restrict__ count_dst) {
    if (count_dst && blockIdx.x == 0 && threadIdx.x < 6) count_dst[threadIdx.x] = count[threadIdx.x];
    const uint32_t n = min(clamp_count(count, cap), out_cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const DevCand c = dc[order[i]];
        fdas_cand o;
        o.k = c.k;
        o.iz = c.iz;
        o.nharm = c.nharm;
        o.r = double(c.k) / (double(c.nharm) * double(cpb));
        o.z = (-zmax + double(c.iz) * dz) / double(c.nharm);
        o.power = c.power;
        o.sigma = float(significance_d(double(c.power), c.nharm));
        out[i] = o;
    }
}

// min(count, cap) records, and the six counter words, written straight into
// page-locked host memory (device aliases), so that the host needs no round
// trip for the count before it can copy the records.
__global__ __launch_bounds__(256) void k_copy_records(const fdas_cand *__restrict__ src,
                                                      const uint32_t *__restrict__ count, uint32_t cap,
                                                      fdas_cand *__restrict__ dst, uint32_t *__restrict__ count_dst) {
    const uint32_t n = clamp_count(count, cap);
    const uint32_t words = n * uint32_t(sizeof(fdas_cand) / 4);
    const uint32_t *__restrict__ s = reinterpret_cast<const uint32_t *>(src);
    uint32_t *__restrict__ d = reinterpret_cast<uint32_t *>(dst);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) d[i] = s[i];
    if (blockIdx.x == 0 && threadIdx.x < 6) count_dst[threadIdx.x] = count[threadIdx.x];
}

}  // namespace

hipError_t launch_copy_records(const fdas_cand *src, const uint32_t *count, uint32_t cap, fdas_cand *dst,
                               uint32_t *count_dst, hipStream_t st) {
    static_assert(sizeof(fdas_cand) % 4 == 0, "whole words");
    const uint64_t words = uint64_t(cap) * (sizeof(fdas_cand) / 4);
    const uint64_t blocks = (words + 255) / 256;
    const unsigned grid = unsigned(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024);
    hipLaunchKernelGGL(k_copy_records, dim3(grid), dim3(256), 0, st, src, count, cap, dst, count_dst);
    return hipGetLastError();
}

// Layout: keys k0, k1 (cap each), values v0, v1 (cap each), then the digit
// counts at the next 16-byte boundary.
size_t cand_sort_scratch_bytes(uint32_t cap) {
    return size_t(cap) * (2 * sizeof(uint64_t) + 2 * sizeof(uint32_t)) + 16 + size_t(RS_DIGITS) * RS_BLOCKS * 4;
}

// Launches: keys (with the first pass's counts), the one-workgroup sort of
// short lists, per radix pass the digit counts (after the first) and the
// scatter (each returns at once for short lists), the public records.
hipError_t launch_finish_candidates(const DevCand *dc, const uint32_t *count, uint32_t cap, void *scratch, int nz,
                                    int64_t nb, int cpb, double zmax, double dz, fdas_cand *out, hipStream_t st,
                                    uint32_t out_cap, uint32_t *count_dst) {
    if (cap == 0) return hipSuccess;
    const uint64_t span = 5 * uint64_t(nb) * uint64_t(nz);  // keys are below this
    int bits = 1;
    while (bits < 64 && (uint64_t(1) << bits) < span) ++bits;
    const int passes = (bits + 7) / 8;
    uint64_t *k0 = static_cast<uint64_t *>(scratch);
    uint64_t *k1 = k0 + cap;
    uint32_t *v0 = reinterpret_cast<uint32_t *>(k1 + cap);
    uint32_t *v1 = v0 + cap;
    uint32_t *hist = reinterpret_cast<uint32_t *>((reinterpret_cast<uintptr_t>(v1 + cap) + 15) & ~uintptr_t(15));
    const uint64_t blocks = (uint64_t(cap) + 255) / 256;
    // Into host memory the records leave at the PCIe rate: with fewer
    // threads than records (about two each for 241 k records) a wave's writes
    // of one record go out while it computes its next significance, instead
    // of every significance first and then all the writes (about 12 us less).
    const uint64_t gmax = count_dst ? 512 : 1024;
    const unsigned grid = unsigned(blocks < gmax ? blocks : gmax);
    hipLaunchKernelGGL(k_cand_keys, dim3(RS_BLOCKS), dim3(RS_THREADS), 0, st, dc, count, cap, nb, nz, k0, v0, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the order ends in v0 after an even number of passes, else in v1
    hipLaunchKernelGGL(k_small_sort, dim3(1), dim3(SMALL_THREADS), 0, st, k0, v0, count, cap,
                       (passes % 2) ? v1 : v0);
    for (int p = 0; p < passes; ++p) {
        if (p > 0)
            hipLaunchKernelGGL(k_rs_hist, dim3(RS_BLOCKS), dim3(RS_THREADS), 0, st, k0, count, cap, 8 * p, hist);
        hipLaunchKernelGGL(k_rs_pass, dim3(RS_BLOCKS), dim3(RS_THREADS), 0, st, k0, v0, count, cap, 8 * p, hist, k1,
                           v1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = k0;
        k0 = k1;
        k1 = tk;
        uint32_t *tv = v0;
        v0 = v1;
        v1 = tv;
    }
    hipLaunchKernelGGL(k_cand_finalize, dim3(grid), dim3(256), 0, st, dc, v0, count, cap, cpb, zmax, dz, out, out_cap,
                       count_dst);
    return hipGetLastError();
}

}  // namespace fdas
