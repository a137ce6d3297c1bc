// Stable radix sort of (uint32 key, int32 value) pairs on the GPU, shared by
// the hierarchy builders.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include "wost_internal.h"

namespace wost {
namespace {

// ---------------------------------------------------------------- radix sort
//
// Stable least-significant-digit radix sort of (uint32 key, int32 value)
// pairs, 8 bits per pass.  A pass: each block counts the digits of its tile
// (kRsTile elements) -> one exclusive scan over the counts laid out digit
// major ([digit][block]), which gives every (digit, block) its first output
// position -> each block walks its tile again in order, 256 elements per
// round, and places each element after the elements of the same digit that
// precede it (ranks inside a wave from ballots over the digit bits, across
// the block's four waves and across rounds from counts in LDS).

constexpr int kRsBits = 8, kRsDigits = 1 << kRsBits;
constexpr int kRsThreads = 256, kRsWaves = kRsThreads / 64, kRsRounds = 16;
constexpr int kRsTile = kRsThreads * kRsRounds;

__global__ __launch_bounds__(kRsThreads) void rs_count(const uint32_t* __restrict__ keys, int n, int shift,
                                                       uint32_t* __restrict__ hist, int nblocks)
{
    __shared__ uint32_t c[kRsDigits];
    c[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        const int i = base + r * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&c[(keys[i] >> shift) & (kRsDigits - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = c[threadIdx.x];
}

// exclusive scan of m counts in one workgroup of 1024 threads: each thread
// sums a contiguous chunk, the chunk sums are scanned in LDS, then each
// thread writes its chunk's exclusive prefixes
__global__ __launch_bounds__(1024) void rs_scan(uint32_t* __restrict__ a, int m, uint32_t* __restrict__ total = nullptr)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int lo = t * per, hi = min(lo + per, m);
    uint32_t sum = 0;
    for (int i = lo; i < hi; ++i) sum += a[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    if (total && t == 1023) *total = part[t];
    uint32_t run = part[t] - sum;
    for (int i = lo; i < hi; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kRsThreads) void rs_scatter(const uint32_t* __restrict__ keys_in,
                                                         const int32_t* __restrict__ vals_in, int n, int shift,
                                                         const uint32_t* __restrict__ offs, int nblocks,
                                                         uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out)
{
    __shared__ uint32_t run[kRsDigits];          // elements of each digit placed so far by this block
    __shared__ uint32_t wc[kRsWaves][kRsDigits];  // this round's count of each digit per wave
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    run[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    const int base = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        for (int w = 0; w < kRsWaves; ++w) wc[w][t] = 0;
        __syncthreads();
        const int i = base + r * kRsThreads + t;
        const bool valid = i < n;
        const uint32_t k = valid ? keys_in[i] : 0u;
        const uint32_t d = (k >> shift) & (kRsDigits - 1);
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRsBits; ++b) {
            const uint64_t m = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t below = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        if (valid && below == 0) wc[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + below;
            for (int w = 0; w < wave; ++w) pos += wc[w][d];
            keys_out[pos] = k;
            vals_out[pos] = vals_in[i];
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kRsWaves; ++w) tot += wc[w][t];
        run[t] += tot;
        __syncthreads();
    }
}

inline int64_t rs_hist_words(int64_t n) { return (int64_t)kRsDigits * std::max<int64_t>((n + kRsTile - 1) / kRsTile, 1); }

// sorts (keys_a, vals_a) into (keys_b, vals_b) by the low `bits` key bits
// (rounded up to whole 8-bit digits, at least one pass); passes alternate
// between the two buffers, and the result always ends in the b buffers.  The
// a buffers are overwritten.
inline int rs_sort_pairs(uint32_t* keys_a, int32_t* vals_a, uint32_t* keys_b, int32_t* vals_b, int n, int bits,
                         uint32_t* hist, hipStream_t s)
{
    if (n <= 0) return WOST_OK;
    const int nblocks = (n + kRsTile - 1) / kRsTile;
    const int m = kRsDigits * nblocks;
    uint32_t* ki = keys_a; int32_t* vi = vals_a; uint32_t* ko = keys_b; int32_t* vo = vals_b;
    const int passes = std::max(1, (bits + kRsBits - 1) / kRsBits);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(rs_count, dim3(nblocks), dim3(kRsThreads), 0, s, ki, n, p * kRsBits, hist, nblocks);
        hipLaunchKernelGGL(rs_scan, dim3(1), dim3(1024), 0, s, hist, m, (uint32_t*)nullptr);
        hipLaunchKernelGGL(rs_scatter, dim3(nblocks), dim3(kRsThreads), 0, s, ki, vi, n, p * kRsBits, hist, nblocks,
                           ko, vo);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    // after an even number of passes the result is back in the a buffers
    if (passes % 2 == 0) {
        if (hipMemcpyAsync(keys_b, keys_a, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(vals_b, vals_a, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return WOST_EHIP;
    }
    return hipGetLastError() == hipSuccess ? WOST_OK : WOST_EHIP;
}


}  // namespace
}  // namespace wost
