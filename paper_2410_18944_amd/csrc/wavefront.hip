// Multi-kernel wavefront solver: the organisation of the paper's own GPU
// system (Sec. 5.1 and Sec. 5.2 "System Integration"), kept as the A/B
// baseline of the persistent walk kernel.  Every walk of the call has its
// state in HBM; a step of all live walks is a sequence of kernels, one per
// stage (closest Dirichlet point, silhouette and radius, guided direction,
// Neumann sample and visibility, source point and visibility, first hit,
// update), each over a compacted queue of walk ids that the previous stage
// appended to.  The guide is evaluated for a whole step queue in one batched
// kernel, optionally on a second stream where it overlaps the geometric
// stages of the other half of the walks.  The host enqueues steps until the
// live queues are empty.
//
// Walks draw the same random words (per walk and step) and run the same
// traversal code as the persistent kernel, so per-walk results agree with it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "walk_state.h"

namespace wost {

// Queues of walk ids (the walk id is also the walk's state slot) and their
// lengths: cnt[0], cnt[1] the live walks at the start of a step (double
// buffered), cnt[2] the walks that step on, cnt[3] Neumann visibility rays,
// cnt[4] source visibility rays.
struct WfQueues {
    uint32_t* act[2];
    uint32_t* step;
    uint32_t* vis;
    uint32_t* svis;
    uint32_t* cnt;
};

// wave-aggregated append of v to q (one atomic per wave)
__device__ __forceinline__ void wf_append(uint32_t* q, uint32_t* cnt, bool app, uint32_t v)
{
    const uint64_t m = __ballot(app);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t b = 0;
    if ((int)threadIdx.x == leader) b = atomicAdd(cnt, (uint32_t)__popcll(m));
    b = __shfl(b, leader);
    if (app) q[b + lane_prefix(m)] = v;
}

__device__ __forceinline__ uint32_t wf_count(const uint32_t* cnt, int k)
{
    return __builtin_amdgcn_readfirstlane(cnt[k]);
}

// per-wave tallies of the solve statistics, added once per wave
__device__ __forceinline__ void wf_tally(unsigned long long* counters, int i, uint32_t v)
{
    const unsigned long long s = wave_sum_u64(v);
    if (threadIdx.x == 0 && s) atomicAdd(counters + i, s);
}

__global__ void wf_set_counts(uint32_t* cnt, uint32_t n_live)
{
    if (threadIdx.x == 0) {
        cnt[0] = n_live;
        cnt[1] = cnt[2] = cnt[3] = cnt[4] = 0;
    }
}

// the queues a step fills start empty
__global__ void wf_begin_step(uint32_t* cnt, int cur)
{
    if (threadIdx.x == 0) {
        cnt[cur ^ 1] = 0;
        cnt[2] = cnt[3] = cnt[4] = 0;
    }
}

// walks [first, first + count) start; their ids fill the first live queue
template <int D>
__global__ __launch_bounds__(64) void wf_init(const WalkParams P, const WfQueues Q, uint32_t first, uint32_t count)
{
    using F = PoolField<D>;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    for (uint32_t j = blockIdx.x * 64 + threadIdx.x; j < count; j += gridDim.x * 64) {
        const uint32_t g = first + j;
        const uint64_t id = g;
        const uint64_t p = id / (uint64_t)P.wpp;
#pragma unroll
        for (int i = 0; i < D; ++i) { pv.f(F::X + i, g) = P.pts[p * D + i]; pv.f(F::NIN + i, g) = 0.f; }
        pv.i(F::ONP, g) = -1;
        pv.f(F::T, g) = 1.f;
        pv.f(F::ACC, g) = 0.f;
        pv.i(F::K, g) = 0;
        pv.u(F::WLO, g) = (uint32_t)id;
        pv.u(F::WHI, g) = (uint32_t)(id >> 32);
        Q.act[0][j] = g;
    }
}

// ---- closest Dirichlet point; epsilon-shell and step-cap termination
template <int D>
__global__ __launch_bounds__(64) void wf_dirichlet(const WalkParams P, const WfQueues Q, int cur)
{
    using F = PoolField<D>;
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, cur);
    uint32_t n_steps = 0, n_walks = 0, n_trunc = 0;
    for (uint32_t b0 = blockIdx.x * 64; b0 < n; b0 += gridDim.x * 64) {
        const uint32_t idx = b0 + lane;
        bool app = false;
        uint32_t g = 0;
        if (idx < n) {
            g = Q.act[cur][idx];
            float x[D], xbar[D];
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
            int prim = -1;
            const float best2 = closest_dirichlet<D>(G.dir, x, INFINITY, xbar, &prim, st);
            ++n_steps;
            const float dD = prim >= 0 ? sqrtf(best2) : INFINITY;
            const int k = pv.i(F::K, g);
            if (dD <= P.eps || k >= P.max_steps) {
                const float gv = prim >= 0 ? field_value<D>(P.g, xbar) : 0.f;
                const float acc = fmaf(pv.f(F::T, g), gv, pv.f(F::ACC, g));
                P.slot_value[g] = acc;
                if (P.slot_steps) P.slot_steps[g] = k + 1;
                ++n_walks;
                if (!(dD <= P.eps)) ++n_trunc;
            } else {
                pv.f(F::DD, g) = dD;
                app = true;
            }
        }
        wf_append(Q.step, Q.cnt + 2, app, g);
    }
    wf_tally(P.counters, 0, n_steps);
    wf_tally(P.counters, 1, n_walks);
    wf_tally(P.counters, 2, n_trunc);
}

// ---- closest silhouette -> star radius; uniform direction
template <int D, bool GUIDED>
__global__ __launch_bounds__(64) void wf_silhouette(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const float area = D == 2 ? 2.f * kPi : 4.f * kPi;
    const uint32_t n = wf_count(Q.cnt, 2);
    for (uint32_t idx = blockIdx.x * 64 + lane; idx < n; idx += gridDim.x * 64) {
        const uint32_t g = Q.step[idx];
        float x[D];
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
        const int onp = pv.i(F::ONP, g);
        const float dD = pv.f(F::DD, g);
        const float best2 = closest_silhouette<D>(G.sil, x, dD * dD, onp, st);
        pv.f(F::R, g) = fmaxf(fminf(dD, sqrtf(best2)), P.r_min);
        pv.f(F::CON, g) = 0.f;
        if constexpr (!GUIDED) {
            const Stream rs = walk_stream(P, g);
            const uint4 wd = rs.block((uint32_t)pv.i(F::K, g), kBlkDir);
            float nu[D];
            uniform_dir<D>(u01(wd.x), u01(wd.y), nu);
            if (onp >= 0) {
                float nin[D];
#pragma unroll
                for (int i = 0; i < D; ++i) nin[i] = pv.f(F::NIN + i, g);
                const float c = dot<D>(nu, nin);
                if (c < 0.f) {
#pragma unroll
                    for (int i = 0; i < D; ++i) nu[i] = fmaf(-2.f * c, nin[i], nu[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) pv.f(F::NU + i, g) = nu[i];
            pv.f(F::W, g) = 1.f;
            pv.f(F::PMIS, g) = 1.f / area;
        }
    }
}

// ---- guided direction: the network over the whole step queue, 64 walks per
// wave on MFMA, then each lane draws from its own mixture
template <int D>
__global__ __launch_bounds__(64) void wf_guide(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    extern __shared__ uint2 s_lds[];
    float* const s_out = (float*)s_lds;
    const int lane = threadIdx.x;
    const int out_stride = guide_out_stride(P.guide);
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const float area = D == 2 ? 2.f * kPi : 4.f * kPi;
    const uint32_t n = wf_count(Q.cnt, 2);
    uint32_t n_bad = 0;
    for (uint32_t b0 = blockIdx.x * 64; b0 < n; b0 += gridDim.x * 64) {
        const uint32_t idx = b0 + lane;
        const bool valid = idx < n;
        const uint32_t g = Q.step[valid ? idx : b0];
        float x[D];
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
        __syncthreads();
        guide_forward_wave<D>(P.guide, x, s_out, lane, out_stride);
        __syncthreads();
        if (valid) {
            const bool onN = pv.i(F::ONP, g) >= 0;
            float nin[D], nu[D], pmis = 1.f / area;
#pragma unroll
            for (int i = 0; i < D; ++i) nin[i] = pv.f(F::NIN + i, g);
            const int k = pv.i(F::K, g);
            const Stream rs = walk_stream(P, g);
            const uint4 wd = rs.block((uint32_t)k, kBlkDir);
            guided_draw<D>(P.guide, s_out + lane * out_stride, rs, (uint32_t)k, wd, onN, nin, nu, &pmis);
            float w = 0.f;
            if (pmis >= 0.f) {
                w = (onN ? 2.f : 1.f) / (area * pmis);
                if (!(w >= 0.f && w < INFINITY)) { ++n_bad; w = 0.f; }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) pv.f(F::NU + i, g) = nu[i];
            pv.f(F::W, g) = w;
            pv.f(F::PMIS, g) = pmis;
        }
    }
    wf_tally(P.counters, 4, n_bad);
}

// ---- Neumann contribution: a point on a Neumann primitive meeting the
// ball, drawn by area; candidates inside the star's half-space queue a
// visibility ray
template <int D>
__global__ __launch_bounds__(64) void wf_neumann(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    const int lane = threadIdx.x;
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, 2);
    for (uint32_t b0 = blockIdx.x * 64; b0 < n; b0 += gridDim.x * 64) {
        const uint32_t idx = b0 + lane;
        bool app = false;
        uint32_t g = 0;
        if (idx < n) {
            g = Q.step[idx];
            float x[D];
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
            const float r = pv.f(F::R, g);
            const uint4 wn = walk_stream(P, g).block((uint32_t)pv.i(F::K, g), kBlkNeu);
            float prob = 0.f;
            const int prim = sample_neumann<D>(G.neu, x, r, u01(wn.x), &prob);
            if (prim >= 0 && prob > 0.f) {
                Prim<D> pr;
                pr.load(G.neu.prims, prim);
                float z[D], dz[D], rho2 = 0.f;
                pr.point(u01(wn.y), u01(wn.z), z);
#pragma unroll
                for (int i = 0; i < D; ++i) { dz[i] = z[i] - x[i]; rho2 = fmaf(dz[i], dz[i], rho2); }
                const float rho = sqrtf(rho2);
                bool ok = rho < r && rho > 0.f;
                const int onp = pv.i(F::ONP, g);
                if (ok && onp >= 0) {
                    float nin[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) nin[i] = pv.f(F::NIN + i, g);
                    if (dot<D>(dz, nin) < -G.tau) ok = false;
                }
                if (ok) {
                    const float4 ex = G.neu.pextra[prim];
                    const float no[3] = {ex.x, ex.y, ex.z};
                    const float hv = neumann_value<D>(P.h, z, no);
                    const float inv_alpha = onp >= 0 ? 2.f : 1.f;
                    pv.f(F::NVAL, g) = green_ball<D>(r, rho) * hv * (ex.w / prob) * inv_alpha;
#pragma unroll
                    for (int i = 0; i < D; ++i) pv.f(F::Z + i, g) = z[i];
                    // the sample's primitive, for its visibility ray (the hit
                    // field is free until the first-hit stage)
                    pv.i(F::HIT, g) = prim;
                    app = true;
                }
            }
        }
        wf_append(Q.vis, Q.cnt + 3, app, g);
    }
}

template <int D>
__global__ __launch_bounds__(64) void wf_neumann_visibility(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, 3);
    for (uint32_t idx = blockIdx.x * 64 + lane; idx < n; idx += gridDim.x * 64) {
        const uint32_t g = Q.vis[idx];
        const int onp = pv.i(F::ONP, g);
        float xo[D], dn[D], l2 = 0.f;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float xi = pv.f(F::X + i, g);
            xo[i] = onp >= 0 ? fmaf(G.tau, pv.f(F::NIN + i, g), xi) : xi;
            dn[i] = pv.f(F::Z + i, g) - xo[i];
            l2 = fmaf(dn[i], dn[i], l2);
        }
        const float len = sqrtf(l2);
#pragma unroll
        for (int i = 0; i < D; ++i) dn[i] /= len;
        if (visible_neumann<D>(G.neu, xo, dn, 0.f, len - G.tau, onp, pv.i(F::HIT, g), st))
            pv.f(F::CON, g) += pv.f(F::NVAL, g);
    }
}

// ---- source contribution: a point of the ball drawn from the radial law of
// its Green's function, kept if visible in the star
template <int D>
__global__ __launch_bounds__(64) void wf_source(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    const int lane = threadIdx.x;
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, 2);
    for (uint32_t b0 = blockIdx.x * 64; b0 < n; b0 += gridDim.x * 64) {
        const uint32_t idx = b0 + lane;
        bool app = false;
        uint32_t g = 0;
        if (idx < n) {
            g = Q.step[idx];
            const Stream rs = walk_stream(P, g);
            const uint32_t k = (uint32_t)pv.i(F::K, g);
            const uint4 a = rs.block(k, kBlkSrc0);
            const uint4 b = rs.block(k, kBlkSrc1);
            float sr;
            if (D == 2) {
                sr = sqrtf(u01(a.x) * u01(a.y));
            } else {
                const float u0 = u01(a.x), u1 = u01(a.y), u2 = u01(a.z);
                sr = fmaxf(fminf(u0, u1), fminf(fmaxf(u0, u1), u2));
            }
            float nu2[D];
            uniform_dir<D>(u01(a.w), u01(b.x), nu2);
            const int onp = pv.i(F::ONP, g);
            float nin[D], x[D];
#pragma unroll
            for (int i = 0; i < D; ++i) { nin[i] = pv.f(F::NIN + i, g); x[i] = pv.f(F::X + i, g); }
            bool ok = sr > 0.f;
            if (ok && onp >= 0 && dot<D>(nu2, nin) <= 0.f) ok = false;
            const float r = pv.f(F::R, g);
            float y[D], l2 = 0.f;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                y[i] = fmaf(sr * r, nu2[i], x[i]);
                const float xo = onp >= 0 ? fmaf(G.tau, nin[i], x[i]) : x[i];
                const float dy = y[i] - xo;
                l2 = fmaf(dy, dy, l2);
            }
            if (ok) {
                const float sterm = (r * r / (2.f * D)) * field_value<D>(P.f, y) * (onp >= 0 ? 2.f : 1.f);
                if (sqrtf(l2) > 0.f) {
                    pv.f(F::SVAL, g) = sterm;
#pragma unroll
                    for (int i = 0; i < D; ++i) pv.f(F::Y + i, g) = y[i];
                    app = true;
                } else {
                    pv.f(F::CON, g) -= sterm;
                }
            }
        }
        wf_append(Q.svis, Q.cnt + 4, app, g);
    }
}

template <int D>
__global__ __launch_bounds__(64) void wf_source_visibility(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, 4);
    for (uint32_t idx = blockIdx.x * 64 + lane; idx < n; idx += gridDim.x * 64) {
        const uint32_t g = Q.svis[idx];
        const int onp = pv.i(F::ONP, g);
        float xo[D], dy[D], l2 = 0.f;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float xi = pv.f(F::X + i, g);
            xo[i] = onp >= 0 ? fmaf(G.tau, pv.f(F::NIN + i, g), xi) : xi;
            dy[i] = pv.f(F::Y + i, g) - xo[i];
            l2 = fmaf(dy[i], dy[i], l2);
        }
        const float len = sqrtf(l2);
#pragma unroll
        for (int i = 0; i < D; ++i) dy[i] /= len;
        if (visible_neumann<D>(G.neu, xo, dy, 0.f, len, onp, -1, st)) pv.f(F::CON, g) -= pv.f(F::SVAL, g);
    }
}

// ---- first hit inside the star; the search runs to r + tau, so a boundary
// point at distance r puts the walker on the boundary, and exits up to tau
// behind the origin count
template <int D>
__global__ __launch_bounds__(64) void wf_hit(const WalkParams P, const WfQueues Q)
{
    using F = PoolField<D>;
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, 2);
    for (uint32_t idx = blockIdx.x * 64 + lane; idx < n; idx += gridDim.x * 64) {
        const uint32_t g = Q.step[idx];
        const int onp = pv.i(F::ONP, g);
        float xo[D], nu[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float xi = pv.f(F::X + i, g);
            xo[i] = onp >= 0 ? fmaf(G.tau, pv.f(F::NIN + i, g), xi) : xi;
            nu[i] = pv.f(F::NU + i, g);
        }
        int hit = -1;
        const float t = ray_neumann<D>(G.neu, xo, nu, pv.f(F::R, g) + G.tau, 0.f, onp, &hit, st,
                                       (NoStat*)nullptr, G.tau);
        pv.f(F::TH, g) = t;
        pv.i(F::HIT, g) = hit;
    }
}

// ---- step update: move, weight, roulette, training record; live walks go
// to the next step's queue
template <int D, bool GUIDED>
__global__ __launch_bounds__(64) void wf_update(const WalkParams P, const WfQueues Q, int cur)
{
    using F = PoolField<D>;
    const int lane = threadIdx.x;
    const DevGeom& G = P.geom;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    const uint32_t n = wf_count(Q.cnt, 2);
    uint32_t n_walks = 0, n_rr = 0, n_rec = 0, n_drop = 0;
    for (uint32_t b0 = blockIdx.x * 64; b0 < n; b0 += gridDim.x * 64) {
        const uint32_t idx = b0 + lane;
        bool live = false, do_rec = false;
        uint32_t g = 0;
        float rec_x[D], rec_nin[D], rec_nu[D], rec_pmis = 0.f, rec_prefix = 0.f, rec_tnext = 0.f;
        if (idx < n) {
            g = Q.step[idx];
            float x[D], nin[D], nu[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                x[i] = pv.f(F::X + i, g);
                nin[i] = pv.f(F::NIN + i, g);
                nu[i] = pv.f(F::NU + i, g);
            }
            int onp = pv.i(F::ONP, g);
            const bool onN = onp >= 0;
            float T = pv.f(F::T, g), acc = pv.f(F::ACC, g);
            int k = pv.i(F::K, g);
            const float r = pv.f(F::R, g), th = pv.f(F::TH, g), w = pv.f(F::W, g);
            const int hp = pv.i(F::HIT, g);
            acc = fmaf(T, pv.f(F::CON, g), acc);
            // a guided draw wasted into the wall (reflection off) ends the walk
            const bool wasted = GUIDED && pv.f(F::PMIS, g) < 0.f;
            bool done = wasted;
            if (wasted) {
                ++k;
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) { rec_x[i] = x[i]; rec_nin[i] = onN ? nin[i] : 0.f; rec_nu[i] = nu[i]; }
                float xo[D];
#pragma unroll
                for (int i = 0; i < D; ++i) xo[i] = onN ? fmaf(G.tau, nin[i], x[i]) : x[i];
                if (hp >= 0) {
                    const float4 ex = G.neu.pextra[hp];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        x[i] = fmaf(th, nu[i], xo[i]);
                        nin[i] = -(i == 0 ? ex.x : (i == 1 ? ex.y : ex.z));
                    }
                    onp = hp;
                } else {
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = fmaf(r, nu[i], xo[i]);
                    onp = -1;
                }
                T *= w;
                ++k;
                if (k >= P.rr_start) {
                    const uint4 wr = walk_stream(P, g).block((uint32_t)k, kBlkNeu);
                    if (u01(wr.w) >= P.rr_q) { done = true; ++n_rr; }
                    else T /= P.rr_q;
                }
#pragma unroll
                for (int i = 0; i < D; ++i) { pv.f(F::X + i, g) = x[i]; pv.f(F::NIN + i, g) = nin[i]; }
                pv.i(F::ONP, g) = onp;
                pv.f(F::T, g) = T;
                rec_pmis = pv.f(F::PMIS, g);
                rec_prefix = acc;
                rec_tnext = T;
                do_rec = GUIDED && P.rec.data != nullptr;
            }
            pv.f(F::ACC, g) = acc;
            pv.i(F::K, g) = k;
            if (done) {
                P.slot_value[g] = acc;
                if (P.slot_steps) P.slot_steps[g] = k;
                ++n_walks;
            } else {
                live = true;
            }
        }
        if constexpr (GUIDED) {
            const uint64_t rm = __ballot(do_rec);
            if (rm) {
                const uint32_t cnt = (uint32_t)__popcll(rm);
                const int leader = __ffsll((unsigned long long)rm) - 1;
                unsigned long long rb = 0;
                if (lane == leader) rb = atomicAdd(P.rec.count, (unsigned long long)cnt);
                const uint32_t blo = __shfl((uint32_t)rb, leader), bhi = __shfl((uint32_t)(rb >> 32), leader);
                rb = ((unsigned long long)bhi << 32) | blo;
                if (do_rec) {
                    const uint64_t row = rb + lane_prefix(rm);
                    if (row < (uint64_t)P.rec.capacity) {
                        float* dst = P.rec.data + row;
                        const int64_t C = P.rec.capacity;
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            dst[(int64_t)i * C] = rec_x[i];
                            dst[(int64_t)(D + i) * C] = rec_nu[i];
                            dst[(int64_t)(2 * D + i) * C] = rec_nin[i];
                        }
                        dst[(int64_t)(3 * D) * C] = rec_pmis;
                        dst[(int64_t)(3 * D + 1) * C] = rec_prefix;
                        dst[(int64_t)(3 * D + 2) * C] = rec_tnext;
                        dst[(int64_t)(3 * D + 3) * C] = __uint_as_float(g);
                        dst[(int64_t)(3 * D + 4) * C] = 0.f;
                        ++n_rec;
                    } else {
                        ++n_drop;
                    }
                }
            }
        }
        wf_append(Q.act[cur ^ 1], Q.cnt + (cur ^ 1), live, g);
    }
    wf_tally(P.counters, 1, n_walks);
    wf_tally(P.counters, 3, n_rr);
    wf_tally(P.counters, 5, n_rec);
    wf_tally(P.counters, 6, n_drop);
}

// one step of a queue set, in three parts: up to the radius, the guided
// direction, and the rest (the guide part may run on another stream)
template <int D, bool GUIDED>
static void enqueue_front(const WalkParams& P, const WfQueues& Q, int cur, int grid, size_t lds_stack, hipStream_t s)
{
    hipLaunchKernelGGL(wf_begin_step, dim3(1), dim3(64), 0, s, Q.cnt, cur);
    hipLaunchKernelGGL(wf_dirichlet<D>, dim3(grid), dim3(64), lds_stack, s, P, Q, cur);
    hipLaunchKernelGGL((wf_silhouette<D, GUIDED>), dim3(grid), dim3(64), lds_stack, s, P, Q);
}

template <int D>
static void enqueue_guide(const WalkParams& P, const WfQueues& Q, int grid, size_t lds_guide, hipStream_t s)
{
    hipLaunchKernelGGL(wf_guide<D>, dim3(grid), dim3(64), lds_guide, s, P, Q);
}

template <int D, bool GUIDED>
static void enqueue_back(const WalkParams& P, const WfQueues& Q, int cur, int grid, size_t lds_stack, bool has_h,
                         bool has_f, hipStream_t s)
{
    if (has_h) {
        hipLaunchKernelGGL(wf_neumann<D>, dim3(grid), dim3(64), 0, s, P, Q);
        hipLaunchKernelGGL(wf_neumann_visibility<D>, dim3(grid), dim3(64), lds_stack, s, P, Q);
    }
    if (has_f) {
        hipLaunchKernelGGL(wf_source<D>, dim3(grid), dim3(64), 0, s, P, Q);
        hipLaunchKernelGGL(wf_source_visibility<D>, dim3(grid), dim3(64), lds_stack, s, P, Q);
    }
    hipLaunchKernelGGL(wf_hit<D>, dim3(grid), dim3(64), lds_stack, s, P, Q);
    hipLaunchKernelGGL((wf_update<D, GUIDED>), dim3(grid), dim3(64), 0, s, P, Q, cur);
}

struct WfLaunch {
    int grid;
    size_t lds_stack, lds_guide;
    bool has_h, has_f;
    hipStream_t s, s2;          // the caller's stream; the inference stream (guided)
    hipEvent_t front[2], inf[2];
};

// One step of every live walk.  With one stream, one queue set runs all its
// stages on the caller's stream.  With the inference stream (guided, two
// streams), the walks are split into two halves with their own queues; the
// network for one half runs on the inference stream while the caller's
// stream runs the other half's geometric stages.
template <int D, bool GUIDED>
static void enqueue_step(const WalkParams& P, const WfQueues* Q, int nq, int cur, const WfLaunch& L)
{
    if (!GUIDED || !L.s2) {
        enqueue_front<D, GUIDED>(P, Q[0], cur, L.grid, L.lds_stack, L.s);
        if (GUIDED) enqueue_guide<D>(P, Q[0], L.grid, L.lds_guide, L.s);
        enqueue_back<D, GUIDED>(P, Q[0], cur, L.grid, L.lds_stack, L.has_h, L.has_f, L.s);
        return;
    }
    for (int h = 0; h < nq; ++h) {
        enqueue_front<D, true>(P, Q[h], cur, L.grid, L.lds_stack, L.s);
        hipEventRecord(L.front[h], L.s);
        hipStreamWaitEvent(L.s2, L.front[h], 0);
        enqueue_guide<D>(P, Q[h], L.grid, L.lds_guide, L.s2);
        hipEventRecord(L.inf[h], L.s2);
    }
    for (int h = 0; h < nq; ++h) {
        hipStreamWaitEvent(L.s, L.inf[h], 0);
        enqueue_back<D, true>(P, Q[h], cur, L.grid, L.lds_stack, L.has_h, L.has_f, L.s);
    }
}

// streams of a guided wavefront solve: 1 (every stage on the caller's
// stream) or 2 (the network on its own stream, overlapping the other half's
// geometric stages)
static int g_wf_streams = 1;

// the inference stream, created once per device at default priority
static hipStream_t inference_stream()
{
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

static inline int64_t wf_align256(int64_t v) { return (v + 255) & ~int64_t(255); }
static inline int wf_words(int dim) { return dim == 2 ? PoolField<2>::WORDS : PoolField<3>::WORDS; }

}  // namespace wost

using namespace wost;

extern "C" int wost_set_wavefront_streams(int32_t n_streams)
{
    if (n_streams != 1 && n_streams != 2) {
        set_error("wost_set_wavefront_streams: 1 or 2 streams");
        return WOST_EINVAL;
    }
    g_wf_streams = n_streams;
    return WOST_OK;
}

extern "C" int64_t wost_solve_wavefront_workspace_bytes(const wost_geom* geom, int64_t n_points, int32_t wpp)
{
    if (!geom || n_points < 0 || wpp <= 0) return -1;
    const int64_t n = n_points * (int64_t)wpp;
    // counters | per-walk values | walk state | 5 queues per half (two halves
    // for guided solves, each sized for its own walks)
    return 256 + wf_align256(n * 4) + wf_align256(n * wf_words(geom->dim) * 4) + 5 * (wf_align256((n + 1) / 2 * 4) +
                                                                                      wf_align256(n / 2 * 4));
}

extern "C" int wost_solve_wavefront(const wost_geom* geom, const wost_problem* pb, const float* pts, int64_t n_points,
                                    int32_t wpp, uint64_t seed, uint64_t walk_offset, const wost_guide* guide,
                                    double* sum, double* sum_sq, int64_t* count, float* walk_value,
                                    int32_t* walk_steps, const wost_records* rec, void* workspace, int64_t ws_bytes,
                                    uint64_t* dev_counters, void* stream)
{
    WalkParams P;
    int rc = prepare_solve("wost_solve_wavefront", geom, pb, pts, n_points, wpp, seed, walk_offset, guide, sum,
                           sum_sq, count, walk_value, walk_steps, rec, workspace, dev_counters, P);
    if (rc != WOST_OK) return rc;
    const int64_t need = wost_solve_wavefront_workspace_bytes(geom, n_points, wpp);
    if (ws_bytes < need) {
        set_error("wost_solve_wavefront: workspace %lld < %lld bytes", (long long)ws_bytes, (long long)need);
        return WOST_ESIZE;
    }
    const int dim = geom->dim;
    const int64_t n = (int64_t)P.n_walks;
    if ((uint64_t)n * (uint64_t)wf_words(dim) >= (1ull << 32)) {
        set_error("wost_solve_wavefront: walk state exceeds 2^32 words; split the call");
        return WOST_EUNSUPPORTED;
    }
    if (P.cost) {
        set_error("wost_solve_wavefront: traversal-cost counters are only kept by wost_solve");
        return WOST_EUNSUPPORTED;
    }
    const bool guided = pb->sampling != WOST_SAMPLING_UNIFORM;
    uint8_t* ws = (uint8_t*)workspace;
    const int64_t vbytes = wf_align256(n * 4);
    P.pool = (uint32_t*)(ws + 256 + vbytes);
    P.pool_total = n;
    P.pool_n = 0;
    uint8_t* qb = ws + 256 + vbytes + wf_align256(n * wf_words(dim) * 4);
    // guided solves on two streams run two halves of the walks
    const bool two = guided && n > 1 && g_wf_streams == 2;
    const int nq = two ? 2 : 1;
    const int64_t cnt_h[2] = {nq == 2 ? (n + 1) / 2 : n, nq == 2 ? n / 2 : 0};
    WfQueues Q[2];
    for (int h = 0; h < nq; ++h) {
        const int64_t qbytes = wf_align256(cnt_h[h] * 4);
        Q[h].act[0] = (uint32_t*)qb;
        Q[h].act[1] = (uint32_t*)(qb + qbytes);
        Q[h].step = (uint32_t*)(qb + 2 * qbytes);
        Q[h].vis = (uint32_t*)(qb + 3 * qbytes);
        Q[h].svis = (uint32_t*)(qb + 4 * qbytes);
        Q[h].cnt = (uint32_t*)(ws + 64 * h);     // queue lengths in the first 256 bytes
        qb += 5 * qbytes;
    }
    hipStream_t s = (hipStream_t)stream;
    WfLaunch L;
    memset(&L, 0, sizeof(L));
    L.s = s;
    L.has_h = P.h.kind != WOST_FIELD_ZERO;
    L.has_f = P.f.kind != WOST_FIELD_ZERO;
    L.lds_stack = sizeof(uint2) * (size_t)geom->stack_need() * kWave;
    L.lds_guide = guided ? sizeof(float) * kWave * (size_t)guide_out_stride(P.guide) : 0;
    // enough waves to keep every CU busy on a long queue; stages read their
    // queue length on the device, so the grid does not follow it
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, (int64_t)walk_num_cu() * 16));
    bool events = false;
    if (two) {
        L.s2 = inference_stream();
        events = L.s2 != nullptr;
        for (int h = 0; h < 2 && events; ++h)
            events = hipEventCreateWithFlags(&L.front[h], hipEventDisableTiming) == hipSuccess &&
                     hipEventCreateWithFlags(&L.inf[h], hipEventDisableTiming) == hipSuccess;
        if (!events) {
            set_error("wost_solve_wavefront: could not create the inference stream or its events");
            return WOST_EHIP;
        }
    }
    const int igrid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, (int64_t)walk_num_cu() * 32));
    int64_t first = 0;
    for (int h = 0; h < nq; ++h) {
        hipLaunchKernelGGL(wf_set_counts, dim3(1), dim3(64), 0, s, Q[h].cnt, (uint32_t)cnt_h[h]);
        if (dim == 2) hipLaunchKernelGGL(wf_init<2>, dim3(igrid), dim3(64), 0, s, P, Q[h], (uint32_t)first, (uint32_t)cnt_h[h]);
        else hipLaunchKernelGGL(wf_init<3>, dim3(igrid), dim3(64), 0, s, P, Q[h], (uint32_t)first, (uint32_t)cnt_h[h]);
        first += cnt_h[h];
    }
    // every step ends a walk whose step count has reached max_steps, so
    // max_steps + 1 steps finish every walk; the live counts are read back
    // every few steps to stop early
    const int64_t max_iter = (int64_t)P.max_steps + 1;
    int cur = 0;
    int rc_loop = WOST_OK;
    for (int64_t it = 0; it < max_iter; ++it) {
        if (dim == 2) {
            if (guided) enqueue_step<2, true>(P, Q, nq, cur, L);
            else enqueue_step<2, false>(P, Q, nq, cur, L);
        } else {
            if (guided) enqueue_step<3, true>(P, Q, nq, cur, L);
            else enqueue_step<3, false>(P, Q, nq, cur, L);
        }
        cur ^= 1;
        if ((it & 7) == 7 || it + 1 == max_iter) {
            uint32_t live[2] = {0, 0};
            bool ok = true;
            for (int h = 0; h < nq && ok; ++h)
                ok = hipMemcpyAsync(&live[h], Q[h].cnt + cur, sizeof(uint32_t), hipMemcpyDeviceToHost, s) == hipSuccess;
            if (!ok || hipStreamSynchronize(s) != hipSuccess) {
                set_error("wost_solve_wavefront: %s", hipGetErrorString(hipGetLastError()));
                rc_loop = WOST_EHIP;
                break;
            }
            if (live[0] + live[1] == 0) break;
        }
    }
    if (events) {
        for (int h = 0; h < 2; ++h) {
            hipEventDestroy(L.front[h]);
            hipEventDestroy(L.inf[h]);
        }
    }
    if (rc_loop != WOST_OK) return rc_loop;
    launch_reduce_points(P, sum, sum_sq, count, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_solve_wavefront: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}
