// Persistent walk-on-stars kernel for gfx950, the per-point FP64 reduction,
// batched geometric queries, and their C ABI (wost_solve, wost_query).
//
// One lane carries one walk.  Each workgroup is a single 64-wide wavefront
// that loops until the global walk counter is exhausted: at the top of every
// step the lanes whose walk finished are refilled together (one atomic per
// wave, lane offsets from mbcnt over the ballot of free lanes), so the wave
// stays full while work remains.  A step visits one star (Sec. 3.2): closest
// Dirichlet point and epsilon-shell test, closest Neumann silhouette -> radius,
// Neumann and source contributions, direction draw, first hit in the star.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

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

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o), hi = __shfl_xor((uint32_t)(v >> 32), o);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

// LDS bytes of one walk workgroup: the traversal stack and the guide's output
// transpose are used in different phases of a step and share the space.  A
// traversal keeps at most one deferred child per internal level of the path it
// is on, so the stack needs (deepest hierarchy's depth) entries; one spare.
static inline size_t walk_lds_bytes(bool guided, int max_depth, int out_stride)
{
    const size_t stack = sizeof(uint2) * (size_t)(max_depth + 1) * kWave;
    const size_t gout = guided ? sizeof(float) * kWave * (size_t)out_stride : 0;
    return stack > gout ? stack : gout;
}

template <int D, bool GUIDED, bool STATS>
__device__ __forceinline__ void walk_body(const WalkParams& P)
{
    // per-query traversal counters (empty structs unless STATS):
    // 0 closest Dirichlet, 1 silhouette, 2 Neumann sample, 3 Neumann
    // visibility, 4 source visibility, 5 first hit
    using S = typename std::conditional<STATS, Stat, NoStat>::type;
    S sq[6];
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    float* const s_out = (float*)s_lds;
    const int out_stride = guide_out_stride(P.guide);
    const DevGeom& G = P.geom;

    bool active = false;
    uint64_t wid = 0;
    Stream rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    rs.p = 0;
    rs.j = 0;
    int k = 0, onp = -1;
    float x[D], nin[D], T = 1.f, acc = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) { x[i] = 0.f; nin[i] = 0.f; }
    bool exhausted = false;
    // the wave's private pool of walk ids [pool_next, pool_end), refilled one
    // chunk at a time from the global counter (one atomic per chunk)
    uint64_t pool_next = 0, pool_end = 0;
    unsigned long long n_steps = 0, n_walks = 0, n_trunc = 0, n_rr = 0, n_bad = 0, n_rec = 0, n_drop = 0;
    const bool has_h = P.h.kind != WOST_FIELD_ZERO;
    const bool has_f = P.f.kind != WOST_FIELD_ZERO;
    const float area = D == 2 ? 2.f * kPi : 4.f * kPi;

    for (;;) {
        // ---- refill free lanes (wave-uniform control flow)
        if (!exhausted) {
            const uint64_t freem = __ballot(!active);
            if (freem) {
                const uint32_t cnt = (uint32_t)__popcll(freem);
                if (pool_next >= pool_end) {
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(P.work, (unsigned long long)P.chunk);
                    const uint32_t blo = __shfl((uint32_t)base, 0), bhi = __shfl((uint32_t)(base >> 32), 0);
                    base = ((unsigned long long)bhi << 32) | blo;
                    pool_next = base;
                    pool_end = base + P.chunk < P.n_walks ? base + P.chunk : P.n_walks;
                    if (base >= P.n_walks) exhausted = true;
                }
                const uint64_t avail = pool_end > pool_next ? pool_end - pool_next : 0;
                if (!active && !exhausted) {
                    const uint64_t slot = lane_prefix(freem);
                    const uint64_t id = pool_next + slot;
                    if (slot < avail) {
                        active = true;
                        wid = id;
                        const uint64_t p = id / (uint64_t)P.wpp;
                        const uint64_t j = id - p * (uint64_t)P.wpp;
                        rs.p = (uint32_t)p;
                        rs.j = (uint32_t)(P.walk_offset + j);
#pragma unroll
                        for (int i = 0; i < D; ++i) { x[i] = P.pts[p * D + i]; nin[i] = 0.f; }
                        k = 0; onp = -1; T = 1.f; acc = 0.f;
                    }
                }
                pool_next += cnt < avail ? cnt : avail;
            }
        }
        if (__ballot(active) == 0) break;
        if constexpr (STATS) {
#pragma unroll
            for (int q = 0; q < 6; ++q) sq[q].step0 = sq[q].nodes;
        }

        // ---- phase A: closest Dirichlet point, epsilon-shell / step-cap termination
        bool stepping = false, finish = false;
        float dD = 0.f;
        if (active) {
            ++n_steps;
            float xbar[D];
            int dp;
            const float d2 = closest_dirichlet<D>(G.dir, x, INFINITY, xbar, &dp, st, &sq[0]);
            dD = sqrtf(d2);
            if (dD <= P.eps || k >= P.max_steps) {
                acc = fmaf(T, field_value<D>(P.g, xbar), acc);
                finish = true;
                if (!(dD <= P.eps)) ++n_trunc;
            } else {
                stepping = true;
            }
        }
        const bool onN = onp >= 0;
        const float inv_alpha = onN ? 2.f : 1.f;

        // ---- phase B+C: direction of the recursive term (guided: wave-wide
        // network evaluation, then each lane draws from its own mixture)
        float nu[D];
        float w = 1.f, pmis = 1.f / area;
        const uint4 wd = rs.block((uint32_t)k, kBlkDir);
        if constexpr (GUIDED) {
            const bool any_step = __ballot(stepping) != 0;
            if (any_step) {
                __syncthreads();
                guide_forward_wave<D>(P.guide, x, s_out, lane, out_stride);
                __syncthreads();
                if (stepping) {
                    guided_draw<D>(P.guide, s_out + lane * out_stride, rs, (uint32_t)k, wd, onN, nin, nu, &pmis);
                    w = inv_alpha / (area * pmis);
                    if (!(w >= 0.f && w < INFINITY)) { ++n_bad; w = 0.f; }
                }
                __syncthreads();
            }
        } else if (stepping) {
            uniform_dir<D>(u01(wd.x), u01(wd.y), nu);
            if (onN) {
                const float c = dot<D>(nu, nin);
                if (c < 0.f) {
#pragma unroll
                    for (int i = 0; i < D; ++i) nu[i] = fmaf(-2.f * c, nin[i], nu[i]);
                }
            }
        }

        // ---- phase D: star radius, Neumann and source terms, first hit
        bool do_rec = false;
        float rec_x[D], rec_nin[D], rec_prefix = 0.f, rec_tnext = 0.f;
        if (stepping) {
            const float dS2 = closest_silhouette<D>(G.sil, x, dD * dD, onp, st, &sq[1]);
            float r = fminf(dD, sqrtf(dS2));
            r = fmaxf(r, P.r_min);
            float contrib = 0.f;
            // ray origin: a walker on the Neumann boundary shoots from a point
            // tau inside along its normal, so every genuine crossing counts
            float xo[D];
#pragma unroll
            for (int i = 0; i < D; ++i) xo[i] = onN ? fmaf(G.tau, nin[i], x[i]) : x[i];
            // Neumann contribution: area-weighted point on a Neumann primitive
            // meeting the ball, kept if it lies in the star
            if (has_h) {
                const uint4 wn = rs.block((uint32_t)k, kBlkNeu);
                float prob;
                const int q = sample_neumann<D>(G.neu, x, r, u01(wn.x), &prob, &sq[2]);
                if (q >= 0 && prob > 0.f) {
                    Prim<D> pr;
                    pr.load(G.neu.prims, q);
                    float z[D], dz[D], rho2 = 0.f;
                    pr.point(u01(wn.y), u01(wn.z), z);
#pragma unroll
                    for (int i = 0; i < D; ++i) { dz[i] = z[i] - x[i]; rho2 = fmaf(dz[i], dz[i], rho2); }
                    const float rho = sqrtf(rho2);
                    bool ok = rho < r && rho > 0.f;
                    if (ok && onN && dot<D>(dz, nin) < -G.tau) ok = false;
                    if (ok) {
                        float dn[D], l2 = 0.f;
#pragma unroll
                        for (int i = 0; i < D; ++i) { dn[i] = z[i] - xo[i]; l2 = fmaf(dn[i], dn[i], l2); }
                        const float len = sqrtf(l2);
#pragma unroll
                        for (int i = 0; i < D; ++i) dn[i] /= len;
                        ok = visible_neumann<D>(G.neu, xo, dn, 0.f, len - G.tau, onp, st, &sq[3]);
                    }
                    if (ok) {
                        const float4 ex = G.neu.pextra[q];
                        const float no[3] = {ex.x, ex.y, ex.z};
                        const float hv = neumann_value<D>(P.h, z, no);
                        contrib += green_ball<D>(r, rho) * hv * (ex.w / prob) * inv_alpha;
                    }
                }
            }
            // source contribution: radius from the radial law of the ball's
            // Green's function, uniform direction, kept if visible in the star
            if (has_f) {
                const uint4 a = rs.block((uint32_t)k, kBlkSrc0);
                const uint4 b = rs.block((uint32_t)k, kBlkSrc1);
                float sr;
                if (D == 2) {
                    sr = sqrtf(u01(a.x) * u01(a.y));
                } else {
                    const float u0 = u01(a.x), u1 = u01(a.y), u2 = u01(a.z);
                    sr = fmaxf(fminf(u0, u1), fminf(fmaxf(u0, u1), u2));
                }
                float nu2[D];
                uniform_dir<D>(u01(a.w), u01(b.x), nu2);
                bool ok = sr > 0.f;
                if (ok && onN && dot<D>(nu2, nin) <= 0.f) ok = false;
                float y[D], dy[D], l2 = 0.f;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    y[i] = fmaf(sr * r, nu2[i], x[i]);
                    dy[i] = y[i] - xo[i];
                    l2 = fmaf(dy[i], dy[i], l2);
                }
                const float len = sqrtf(l2);
                if (ok && len > 0.f) {
#pragma unroll
                    for (int i = 0; i < D; ++i) dy[i] /= len;
                    ok = visible_neumann<D>(G.neu, xo, dy, 0.f, len, onp, st, &sq[4]);
                }
                if (ok) contrib -= (r * r / (2.f * D)) * field_value<D>(P.f, y) * inv_alpha;
            }
            acc = fmaf(T, contrib, acc);
#pragma unroll
            for (int i = 0; i < D; ++i) { rec_x[i] = x[i]; rec_nin[i] = onN ? nin[i] : 0.f; }
            // first hit inside the star
            int hp;
            // the search runs to r + tau, so a boundary point at distance r
            // (a silhouette point straight ahead) puts the walker on the
            // boundary, and exits up to tau behind the origin count (the
            // origin is then on the boundary up to rounding)
            const float t = ray_neumann<D>(G.neu, xo, nu, r + G.tau, 0.f, onp, &hp, st, &sq[5], G.tau);
            if (hp >= 0) {
#pragma unroll
                for (int i = 0; i < D; ++i) x[i] = fmaf(t, nu[i], xo[i]);
                // the walk's side of a Neumann primitive is the domain, so its
                // normal toward the walk is -n_out (a first hit seen from
                // inside is always an exit, nu . n_out > 0)
                const float4 ex = G.neu.pextra[hp];
#pragma unroll
                for (int i = 0; i < D; ++i) nin[i] = -(i == 0 ? ex.x : (i == 1 ? ex.y : ex.z));
                onp = hp;
            } else {
                // the segment from the ray's origin to this point crosses no
                // boundary, so the walker stays inside; stepping from x itself
                // could leave the domain by up to tau along a grazing ray
#pragma unroll
                for (int i = 0; i < D; ++i) x[i] = fmaf(r, nu[i], xo[i]);
                onp = -1;
            }
            T *= w;
            ++k;
            // Russian roulette for the next star (played with that step's word)
            if (k >= P.rr_start) {
                const uint4 wr = rs.block((uint32_t)k, kBlkNeu);
                if (u01(wr.w) >= P.rr_q) { finish = true; ++n_rr; }
                else T /= P.rr_q;
            }
            rec_prefix = acc;
            rec_tnext = T;
            do_rec = GUIDED && P.rec.data != nullptr;
        }

        // wave-level iterations of each query this step: the wave runs a
        // traversal loop for as long as its slowest lane
        if constexpr (STATS) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const uint32_t m = wave_max_u32(sq[q].nodes - sq[q].step0);
                if (lane == 0) sq[q].witer += m;
            }
        }

        // ---- phase E: training record append (one atomic per wave)
        if constexpr (GUIDED) {
            const uint64_t rm = __ballot(do_rec);
            if (rm) {
                const uint32_t cnt = (uint32_t)__popcll(rm);
                const int leader = __ffsll((unsigned long long)rm) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(P.rec.count, (unsigned long long)cnt);
                const uint32_t blo = __shfl((uint32_t)base, leader), bhi = __shfl((uint32_t)(base >> 32), leader);
                base = ((unsigned long long)bhi << 32) | blo;
                if (do_rec) {
                    const uint64_t row = base + lane_prefix(rm);
                    if (row < (uint64_t)P.rec.capacity) {
                        float* dst = P.rec.data + row;
                        const int64_t C = P.rec.capacity;
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            dst[(int64_t)i * C] = rec_x[i];
                            dst[(int64_t)(D + i) * C] = nu[i];
                            dst[(int64_t)(2 * D + i) * C] = rec_nin[i];
                        }
                        dst[(int64_t)(3 * D) * C] = pmis;
                        dst[(int64_t)(3 * D + 1) * C] = rec_prefix;
                        dst[(int64_t)(3 * D + 2) * C] = rec_tnext;
                        dst[(int64_t)(3 * D + 3) * C] = __uint_as_float((uint32_t)wid);
                        dst[(int64_t)(3 * D + 4) * C] = 0.f;
                        ++n_rec;
                    } else {
                        ++n_drop;
                    }
                }
            }
        }

        if (finish) {
            ++n_walks;
            P.slot_value[wid] = acc;
            if (P.slot_steps) P.slot_steps[wid] = k + (stepping ? 0 : 1);
            active = false;
        }
    }
    // ---- statistics: one atomic per wave and counter
    if constexpr (STATS) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const unsigned long long a = wave_sum_u64(sq[q].nodes), b = wave_sum_u64(sq[q].prims);
            if (lane == 0) {
                atomicAdd(P.cost + 2 * q, a);
                atomicAdd(P.cost + 2 * q + 1, b);
                atomicAdd(P.cost + 12 + q, sq[q].witer);
            }
        }
    }
    const unsigned long long vals[7] = {n_steps, n_walks, n_trunc, n_rr, n_bad, n_rec, n_drop};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const unsigned long long sm = wave_sum_u64(vals[i]);
        if (lane == 0 && sm) atomicAdd(P.counters + i, sm);
    }
}

// 2D: at least four resident waves per SIMD (<= 128 VGPRs) keeps every
// variant free of spills.  3D keeps the compiler's choice: its guide encoder
// (16 levels x 8 corners) would spill under that bound.
template <bool GUIDED, bool STATS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void walk_kernel2(const WalkParams P)
{
    walk_body<2, GUIDED, STATS>(P);
}

template <bool GUIDED, bool STATS>
__global__ __launch_bounds__(64) void walk_kernel3(const WalkParams P)
{
    walk_body<3, GUIDED, STATS>(P);
}

__global__ void zero_u64(unsigned long long* p, int n)
{
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Per-point FP64 sums over contiguous walk slots; one wave per point, fixed
// reduction order (deterministic).
__global__ __launch_bounds__(256) void reduce_points(const float* __restrict__ slot, int64_t n_points, int32_t wpp,
                                                     double* sum, double* sum_sq, int64_t* count)
{
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n_points) return;
    double s = 0.0, q = 0.0;
    const float* v = slot + p * (int64_t)wpp;
    for (int j = lane; j < wpp; j += 64) {
        const double t = (double)v[j];
        s += t;
        q = fma(t, t, q);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o);
        q += __shfl_xor(q, o);
    }
    if (lane == 0) {
        sum[p] += s;
        sum_sq[p] += q;
        count[p] += wpp;
    }
}

template <int D>
__global__ __launch_bounds__(64) void query_kernel(const DevGeom G, const float* pts, int64_t n, float* d_dir,
                                                   float* xbar, float* d_sil, const float* ray_dir,
                                                   const float* ray_tmax, float* ray_t, int32_t* ray_prim)
{
    __shared__ uint2 s_stack[kMaxStack * kWave];
    const int lane = threadIdx.x;
    const LdsStack st{&s_stack[lane]};
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    if (i >= n) return;
    float x[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = pts[i * D + c];
    if (d_dir) {
        float xb[D];
        int pr;
        const float d2 = closest_dirichlet<D>(G.dir, x, INFINITY, xb, &pr, st);
        d_dir[i] = pr >= 0 ? sqrtf(d2) : INFINITY;
        if (xbar) {
#pragma unroll
            for (int c = 0; c < D; ++c) xbar[i * D + c] = pr >= 0 ? xb[c] : INFINITY;
        }
    }
    if (d_sil) d_sil[i] = sqrtf(closest_silhouette<D>(G.sil, x, INFINITY, -1, st));
    if (ray_dir && ray_t) {
        float nu[D];
#pragma unroll
        for (int c = 0; c < D; ++c) nu[c] = ray_dir[i * D + c];
        int hp;
        const float t = ray_neumann<D>(G.neu, x, nu, ray_tmax[i], 0.f, -1, &hp, st);
        ray_t[i] = t;
        if (ray_prim) ray_prim[i] = hp >= 0 ? G.neu.orig[hp] : -1;
    }
}

static int g_num_cu = 0;

static int num_cu()
{
    if (g_num_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            g_num_cu = v;
        else
            g_num_cu = 256;
    }
    return g_num_cu;
}

static int g_waves_per_cu = 0;   // 0: resident capacity of the launched variant
static unsigned long long* g_cost = nullptr;

static bool copy_field(const wost_field& in, int dim, FieldDev& out, const char* name)
{
    memset(&out, 0, sizeof(out));
    out.kind = in.kind;
    out.n = in.n;
    if (in.kind < WOST_FIELD_ZERO || in.kind > WOST_FIELD_GAUSS_SUM) {
        set_error("wost_solve: field %s has unknown kind %d", name, in.kind);
        return false;
    }
    int nvals = 0;
    if (in.kind == WOST_FIELD_CONST) nvals = 1;
    if (in.kind == WOST_FIELD_GAUSS_SUM) {
        if (in.n < 0 || in.n > WOST_MAX_GAUSS) { set_error("wost_solve: field %s: 0..%d Gaussians", name, WOST_MAX_GAUSS); return false; }
        nvals = in.n * (2 + dim);
    }
    if (nvals > 0) {
        if (!in.params) { set_error("wost_solve: field %s needs params", name); return false; }
        memcpy(out.p, in.params, sizeof(float) * nvals);
    }
    if ((in.kind == WOST_FIELD_EXP_SIN || in.kind == WOST_FIELD_RE_Z3) && dim != 2) {
        set_error("wost_solve: field %s kind %d is two-dimensional", name, in.kind);
        return false;
    }
    return true;
}

}  // namespace wost

using namespace wost;

extern "C" int64_t wost_solve_workspace_bytes(const wost_geom* geom, int64_t n_points, int32_t wpp)
{
    if (!geom || n_points < 0 || wpp <= 0) return -1;
    return 256 + ((n_points * (int64_t)wpp * 4 + 255) & ~int64_t(255));
}

extern "C" int wost_set_cost_counters(uint64_t* dev_counters18)
{
    g_cost = (unsigned long long*)dev_counters18;
    return WOST_OK;
}

extern "C" int wost_set_launch(int32_t waves_per_cu)
{
    if (waves_per_cu < 0 || waves_per_cu > 64) { set_error("wost_set_launch: waves_per_cu in [0, 64]"); return WOST_EINVAL; }
    g_waves_per_cu = waves_per_cu;
    return WOST_OK;
}

extern "C" int wost_solve(const wost_geom* geom, const wost_problem* pb, const float* pts, int64_t n_points,
                          int32_t wpp, uint64_t seed, uint64_t walk_offset, const wost_guide* guide, double* sum,
                          double* sum_sq, int64_t* count, float* walk_value, int32_t* walk_steps,
                          const wost_records* rec, void* workspace, int64_t ws_bytes, uint64_t* dev_counters,
                          void* stream)
{
    if (!geom || !pb || !pts || !sum || !sum_sq || !count || !workspace || !dev_counters) {
        set_error("wost_solve: NULL argument");
        return WOST_EINVAL;
    }
    if (!geom->dev) { set_error("wost_solve: geometry not uploaded"); return WOST_ESTATE; }
    if (geom->n_dir == 0) { set_error("wost_solve: the boundary has no Dirichlet part (walks never end)"); return WOST_EINVAL; }
    if (n_points <= 0 || wpp <= 0) { set_error("wost_solve: n_points and wpp must be positive"); return WOST_EINVAL; }
    if (n_points > 0xFFFFFFFFll || walk_offset + (uint64_t)wpp > 0xFFFFFFFFull) {
        set_error("wost_solve: point index and walk index must fit 32 bits");
        return WOST_EUNSUPPORTED;
    }
    const int64_t need = wost_solve_workspace_bytes(geom, n_points, wpp);
    if (ws_bytes < need) { set_error("wost_solve: workspace %lld < %lld bytes", (long long)ws_bytes, (long long)need); return WOST_ESIZE; }
    if (!(pb->eps > 0.f) || pb->max_steps < 0 || !(pb->rr_q > 0.f && pb->rr_q <= 1.f) || pb->r_min < 0.f) {
        set_error("wost_solve: need eps > 0, max_steps >= 0, 0 < rr_q <= 1, r_min >= 0");
        return WOST_EINVAL;
    }
    const bool guided = pb->sampling != WOST_SAMPLING_UNIFORM;
    if (pb->sampling < 0 || pb->sampling > WOST_SAMPLING_GUIDED_ONLY) { set_error("wost_solve: unknown sampling mode"); return WOST_EINVAL; }
    if (guided != (guide != nullptr)) { set_error("wost_solve: guide must be given iff sampling is not UNIFORM"); return WOST_EINVAL; }
    if (pb->sampling == WOST_SAMPLING_MIS_FIXED && !(pb->c_fixed >= 0.f && pb->c_fixed <= 1.f)) {
        set_error("wost_solve: c_fixed must be in [0, 1]");
        return WOST_EINVAL;
    }
    WalkParams P;
    memset(&P, 0, sizeof(P));
    P.geom = geom->devgeom();
    const int dim = geom->dim;
    if (!copy_field(pb->g, dim, P.g, "g") || !copy_field(pb->h, dim, P.h, "h") || !copy_field(pb->f, dim, P.f, "f"))
        return WOST_EINVAL;
    if (P.h.kind != WOST_FIELD_ZERO && geom->n_neu == 0) P.h.kind = WOST_FIELD_ZERO;
    P.eps = pb->eps;
    P.r_min = pb->r_min > 0.f ? pb->r_min : pb->eps;
    P.rr_q = pb->rr_q;
    P.max_steps = pb->max_steps;
    P.rr_start = pb->rr_start;
    P.sampling = pb->sampling;
    P.c_fixed = pb->c_fixed;
    P.reflect = pb->reflect;
    P.pts = pts;
    P.n_points = n_points;
    P.wpp = wpp;
    P.key0 = (uint32_t)seed;
    P.key1 = (uint32_t)(seed >> 32);
    P.walk_offset = walk_offset;
    P.n_walks = (uint64_t)n_points * (uint64_t)wpp;
    uint8_t* ws = (uint8_t*)workspace;
    P.work = (unsigned long long*)ws;
    P.slot_value = walk_value ? walk_value : (float*)(ws + 256);
    P.slot_steps = walk_steps;
    P.counters = (unsigned long long*)dev_counters;
    P.cost = g_cost;
    if (guided) {
        int rc = guide_prepare(guide, dim, P.guide);
        if (rc != WOST_OK) return rc;
        P.guide.sampling = pb->sampling;
        P.guide.c_fixed = pb->c_fixed;
        P.guide.reflect = pb->reflect;
    }
    if (rec) {
        if (!guided) { set_error("wost_solve: training records need a guided sampling mode"); return WOST_EINVAL; }
        if (!rec->data || !rec->count || rec->capacity < 0) { set_error("wost_solve: bad record buffer"); return WOST_EINVAL; }
        P.rec.data = rec->data;
        P.rec.capacity = rec->capacity;
        P.rec.count = (unsigned long long*)rec->count;
    }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, P.work, 1);
    using WalkFn = void (*)(const WalkParams);
    WalkFn fn;
    if (dim == 2) {
        if (P.cost) fn = guided ? walk_kernel2<true, true> : walk_kernel2<false, true>;
        else fn = guided ? walk_kernel2<true, false> : walk_kernel2<false, false>;
    } else {
        if (P.cost) fn = guided ? walk_kernel3<true, true> : walk_kernel3<false, true>;
        else fn = guided ? walk_kernel3<true, false> : walk_kernel3<false, false>;
    }
    const size_t lds = walk_lds_bytes(guided, geom->max_depth, guide_out_stride(P.guide));
    int per_cu = g_waves_per_cu;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, lds) != hipSuccess || nb < 1) nb = 8;
        per_cu = nb;
    }
    const uint64_t waves_needed = (P.n_walks + 63) / 64;
    const uint64_t cap = (uint64_t)num_cu() * (uint64_t)per_cu;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(waves_needed, cap));
    // about eight reservations per wave over the whole call, at least one lane's worth each
    P.chunk = std::max<uint64_t>(64, std::min<uint64_t>(4096, P.n_walks / ((uint64_t)grid * 8)));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64), lds, s, P);
    const int rgrid = (int)((n_points + 3) / 4);
    hipLaunchKernelGGL(reduce_points, dim3(rgrid), dim3(256), 0, s, P.slot_value, n_points, wpp, sum, sum_sq, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_solve: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_query(const wost_geom* geom, const float* pts, int64_t n, float* d_dir, float* xbar, float* d_sil,
                          const float* ray_dir, const float* ray_tmax, float* ray_t, int32_t* ray_prim, void* stream)
{
    if (!geom) { set_error("wost_query: NULL geometry"); return WOST_EINVAL; }
    if (!geom->dev) { set_error("wost_query: geometry not uploaded"); return WOST_ESTATE; }
    if (n < 0) { set_error("wost_query: n < 0"); return WOST_EINVAL; }
    if (n > 0 && !pts) { set_error("wost_query: NULL points"); return WOST_EINVAL; }
    if ((ray_dir != nullptr) != (ray_t != nullptr) || (ray_dir && !ray_tmax)) {
        set_error("wost_query: ray_dir, ray_tmax and ray_t go together");
        return WOST_EINVAL;
    }
    if (n == 0) return WOST_OK;
    const DevGeom G = geom->devgeom();
    hipStream_t s = (hipStream_t)stream;
    const int grid = (int)((n + 63) / 64);
    if (geom->dim == 2)
        hipLaunchKernelGGL(query_kernel<2>, dim3(grid), dim3(64), 0, s, G, pts, n, d_dir, xbar, d_sil, ray_dir, ray_tmax, ray_t, ray_prim);
    else
        hipLaunchKernelGGL(query_kernel<3>, dim3(grid), dim3(64), 0, s, G, pts, n, d_dir, xbar, d_sil, ray_dir, ray_tmax, ray_t, ray_prim);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_query: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}
