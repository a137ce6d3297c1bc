// Walk state shared by the persistent walk kernel and the multi-kernel
// wavefront solver: launch parameters, the field-major walk-state layout,
// per-walk random streams and wave-level helpers.
#pragma once

#include <hip/hip_runtime.h>

#include "geom_device.h"
#include "guide_device.h"
#include "guide_internal.h"
#include "walk_common.h"

namespace wost {

struct WalkParams {
    DevGeom geom;
    FieldDev g, h, f;
    float eps, r_min, rr_q;
    int32_t max_steps, rr_start;
    int32_t sampling;
    float c_fixed;
    int32_t reflect;
    const float* pts;
    int64_t n_points;
    int32_t wpp;
    uint32_t key0, key1;
    uint64_t walk_offset;
    uint64_t n_walks;
    float* slot_value;
    int32_t* slot_steps;
    unsigned long long* work;       // global walk counter
    uint64_t chunk;                 // walks a wave reserves per atomic
    unsigned long long* counters;   // 8 stats
    unsigned long long* cost;       // 12 traversal counters (statistics variant only)
    GuideDev guide;
    RecDev rec;
    uint32_t* pool;                 // walk pools: PoolField<D>::WORDS arrays of pool_total words
    int64_t pool_total;             // slots over all waves (grid * pool_n)
    int32_t pool_n;                 // slots per wave (multiple of 64)
    int32_t* lists;                 // 4 work lists of pool_n entries per wave
    int32_t refill_batch;           // finished lanes that wait for a joint refill
};

__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o), hi = __shfl_xor((uint32_t)(v >> 32), o);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

enum : int { ST_EMPTY = 0, ST_ACTIVE = 1, ST_STEP = 2, ST_DONE = 3 };

template <int D>
struct PoolField {
    static constexpr int X = 0, NIN = D, NU = 2 * D, Z = 3 * D, Y = 4 * D;
    static constexpr int T = 5 * D, ACC = T + 1, DD = T + 2, R = T + 3, W = T + 4, PMIS = T + 5, CON = T + 6,
                         NVAL = T + 7, SVAL = T + 8, TH = T + 9, K = T + 10, ONP = T + 11, HIT = T + 12,
                         STAT = T + 13, WLO = T + 14, WHI = T + 15;
    static constexpr int WORDS = T + 16;
};

// Field-major storage (field f of global slot g at pool[f * total + g]):
// the finalize pass and the start of every phase touch consecutive slots, so
// a field access of the wave is one contiguous 256-byte block.  32-bit word
// offsets (fields * slots < 2^32, checked on the host) keep each access one
// VGPR offset from a scalar base.
template <int D>
struct PoolView {
    uint32_t* base;
    uint32_t total;
    __device__ __forceinline__ float& f(int fld, uint32_t g) const { return ((float*)base)[(uint32_t)fld * total + g]; }
    __device__ __forceinline__ int32_t& i(int fld, uint32_t g) const { return ((int32_t*)base)[(uint32_t)fld * total + g]; }
    __device__ __forceinline__ uint32_t& u(int fld, uint32_t g) const { return base[(uint32_t)fld * total + g]; }
    __device__ __forceinline__ uint64_t wid(uint32_t g) const
    {
        return (uint64_t)u(PoolField<D>::WLO, g) | ((uint64_t)u(PoolField<D>::WHI, g) << 32);
    }
};

__device__ __forceinline__ uint64_t wave_uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ Stream walk_stream(const WalkParams& P, uint64_t wid)
{
    Stream rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    const uint64_t p = wid / (uint64_t)P.wpp;
    rs.p = (uint32_t)p;
    rs.j = (uint32_t)(P.walk_offset + (wid - p * (uint64_t)P.wpp));
    return rs;
}

// memory written by one lane of the wave becomes visible to the others
__device__ __forceinline__ void wave_sync()
{
    __threadfence_block();
    __syncthreads();
}

// Host side, defined with the persistent solver: argument checks and the
// launch parameters both solvers share, and the per-point FP64 reduction of
// the per-walk values.
int prepare_solve(const char* who, const wost_geom* geom, const wost_problem* pb, const float* pts, int64_t n_points,
                  int32_t wpp, uint64_t seed, uint64_t walk_offset, const wost_guide* guide, double* sum,
                  double* sum_sq, int64_t* count, float* walk_value, int32_t* walk_steps, const wost_records* rec,
                  void* workspace, uint64_t* dev_counters, WalkParams& P);
void launch_reduce_points(const WalkParams& P, double* sum, double* sum_sq, int64_t* count, hipStream_t s);
int walk_num_cu();

}  // namespace wost
