// Persistent walk-on-stars kernel for gfx950, the per-point FP64 reduction,
// batched geometric queries, and their C ABI (wost_solve, wost_query,
// wost_neumann_sample).
//
// Each workgroup is a single 64-wide wavefront that owns a pool of walk
// slots (structure of arrays in the caller's workspace) and loops until the
// global walk counter is exhausted.  A round advances every live walk of the
// pool by one star (Sec. 3.2), one query at a time: step update and refill
// of empty slots (chunks of walk ids from one atomic per wave, lane offsets
// from mbcnt over the ballot), closest Dirichlet point and epsilon-shell
// test, closest Neumann silhouette -> radius, guided direction (network on
// MFMA for 64 walks at a time), Neumann sample and its visibility, source
// point and its visibility, first hit in the star.  Inside a query phase a
// lane whose traversal has finished takes the next walk of that phase's
// list, so the wave does not wait for its slowest lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "geom_device.h"
#include "guide_device.h"
#include "guide_internal.h"
#include "walk_common.h"
#include "walk_state.h"

namespace wost {

// LDS bytes of one walk workgroup: the traversal stack and the guide's output
// transpose are used in different phases of a step and share the space.  A
// traversal defers at most three children per level of the path it is on;
// the builder reports the entries the deepest hierarchy needs.
static inline size_t walk_lds_bytes(bool guided, int stack_entries, int out_stride)
{
    const size_t stack = sizeof(uint2) * (size_t)stack_entries * kWave;
    const size_t gout = guided ? sizeof(float) * kWave * (size_t)out_stride : 0;
    return stack > gout ? stack : gout;
}

// ---------------------------------------------------------------- walk pool
//
// Each wave owns N walk slots, kept as structure of arrays in the caller's
// workspace.  A round moves
// every live walk of the pool one star forward, phase by phase: closest
// Dirichlet point, closest silhouette (star radius, uniform direction), guide
// evaluation and guided direction in full 64-walk chunks, Neumann sample and
// its visibility, source point and its visibility, first hit, then the step
// update.  Inside a traversal phase a lane whose query has finished takes the
// next walk of that phase's list at once, so the wave does not wait for its
// slowest lane; lanes of a phase all run the same query code.  Phases whose
// query length can be predicted from the pool (closest Dirichlet point in 3D,
// closest silhouette) hand out their longest queries first.  Once the wave
// can start no new walks it moves its live walks to the front of the pool, so
// the last rounds scan only the occupied slots.

// Lanes that have finished their query wait until at least this many are
// waiting (or no lane is still traversing) before they store results and
// take new work together: finishing and refilling is far more code than one
// traversal iteration, and run for a handful of lanes at a time it would cost
// nearly as much as for all 64.
// Default per dimension (2D, 3D): 3D traversal iterations are long chains of
// dependent fetches from beyond L2, so lanes idling until a large batch has
// finished cost more there (measured: 2D best at 32, 3D at 8).
constexpr int kDefaultRefillBatch[2] = {32, 8};
static int g_refill_batch = 0;   // 0: the default of the solve's dimension

// One traversal phase over list[0, n) with refill from the list: init(slot)
// loads a walk's query, step() advances it by one node and returns true when
// done, finish(slot) stores the result and returns true to append the slot
// to `out` (if given).  `out_n` and the loop counters stay wave-uniform.
template <class Init, class Step, class Finish>
__device__ __forceinline__ void run_phase(const int32_t* list, int n, int32_t* out, int& out_n, int lane, int batch,
                                          unsigned long long& iters, Init&& init, Step&& step, Finish&& finish)
{
    int slot = -1;
    bool waiting = false;
    int next = n < kWave ? n : kWave;
    if (lane < n) {
        slot = list[lane];
        init(slot);
    }
    for (;;) {
        const bool running = slot >= 0 && !waiting;
        const uint64_t run_m = __ballot(running);
        const uint64_t wait_m = __ballot(waiting);
        if (run_m == 0 && wait_m == 0) break;
        if (run_m) {
            ++iters;
            if (running) waiting = step();
        }
        const uint64_t w2 = __ballot(waiting);
        if (w2 == 0) continue;
        const uint64_t r2 = __ballot(slot >= 0 && !waiting);
        if (__popcll(w2) < batch && r2 != 0) continue;
        // finish and refill every waiting lane
        bool app = false;
        if (waiting) app = finish(slot);
        if (out) {
            const uint64_t m = __ballot(app);
            if (m) {
                if (app) out[out_n + (int)lane_prefix(m)] = slot;
                out_n += __popcll(m);
            }
        }
        if (waiting) {
            const int i = next + (int)lane_prefix(w2);
            slot = i < n ? list[i] : -1;
            waiting = false;
            if (slot >= 0) init(slot);
        }
        next += __popcll(w2);
    }
}

// List the pool slots selected by in(g) in two groups: first those whose
// key(g) is at least the mean key of the selected slots, then the rest, each
// group in slot order.  The keys predict how long a walk's next query runs;
// a phase hands its list out in order, so long queries start early instead of
// trailing at the end of the phase while the other lanes idle, and
// neighbouring lanes read neighbouring slots.  Returns the list length.
template <class In, class Key>
__device__ __forceinline__ int list_long_first(int32_t* L, int N, uint32_t base, int lane, In&& in, Key&& key)
{
    float ksum = 0.f;
    int kn = 0;
    for (int c0 = 0; c0 < N; c0 += kWave) {
        const uint32_t g = base + c0 + lane;
        if (in(g)) { ksum += key(g); ++kn; }
    }
    // each slot is classified by the same lane in both passes, so a lane's
    // own rounding of the mean cannot drop or repeat a slot
    const float thr = wave_sum_f(ksum) / fmaxf((float)wave_sum_i(kn), 1.f);
    int n = 0;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        for (int c0 = 0; c0 < N; c0 += kWave) {
            const int li = c0 + lane;
            const uint32_t g = base + li;
            bool sel = in(g);
            if (sel) {
                const bool longq = key(g) >= thr;
                sel = pass == 0 ? longq : !longq;
            }
            const uint64_t m = __ballot(sel);
            if (sel) L[n + (int)lane_prefix(m)] = li;
            n += __popcll(m);
        }
    }
    return n;
}

template <int D, bool GUIDED, bool STATS>
__device__ __forceinline__ void walk_body(const WalkParams& P)
{
    using F = PoolField<D>;
    // per-query traversal counters (empty structs unless STATS):
    // 0 closest Dirichlet, 1 silhouette, 2 Neumann sample, 3 Neumann
    // visibility, 4 source visibility, 5 first hit
    using S = typename std::conditional<STATS, Stat, NoStat>::type;
    S sq[6];
    unsigned long long witer[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    extern __shared__ uint2 s_lds[];
    const int lane = threadIdx.x;
    const LdsStack st{&s_lds[lane]};
    float* const s_out = (float*)s_lds;
    const int out_stride = guide_out_stride(P.guide);
    const DevGeom& G = P.geom;
    const int N = P.pool_n;
    const uint32_t base = (uint32_t)blockIdx.x * (uint32_t)N;
    const PoolView<D> pv{P.pool, (uint32_t)P.pool_total};
    int32_t* const L_act = P.lists + (int64_t)blockIdx.x * 4 * N;
    int32_t* const L_step = L_act + N;
    int32_t* const L_vis = L_act + 2 * N;
    int32_t* const L_svis = L_act + 3 * N;
    const bool has_h = P.h.kind != WOST_FIELD_ZERO;
    const bool has_f = P.f.kind != WOST_FIELD_ZERO;
    const float area = D == 2 ? 2.f * kPi : 4.f * kPi;
    uint32_t n_steps = 0, n_walks = 0, n_trunc = 0, n_rr = 0, n_bad = 0, n_rec = 0, n_drop = 0;
    bool exhausted = false;
    // the wave's private range of walk ids [pool_next, pool_end), refilled one
    // chunk at a time from the global counter (one atomic per chunk)
    uint64_t pool_next = 0, pool_end = 0;
    int dummy_n = 0;
    const int batch = P.refill_batch;

    for (int c = lane; c < N; c += kWave) pv.i(F::STAT, base + c) = ST_EMPTY;
    wave_sync();
    int Nn = N;  // scanned prefix of the pool (shrinks once no new walks come)

    for (;;) {
        // ---- step update of last round's walks, retirement, refill
        int n_act = 0;
        for (int c0 = 0; c0 < Nn; c0 += kWave) {
            const int li = c0 + lane;
            const uint32_t g = base + li;
            int stt = pv.i(F::STAT, g);
            bool do_rec = false;
            float rec_x[D], rec_nin[D], rec_nu[D], rec_pmis = 0.f, rec_prefix = 0.f, rec_tnext = 0.f;
            uint64_t wid = 0;
            if (stt == ST_STEP) {
                wid = pv.wid(g);
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
                // a guided draw wasted into the wall (reflection off): this
                // star's terms count, its recursive term is zero, the walk ends
                const bool wasted = GUIDED && pv.f(F::PMIS, g) < 0.f;
                if (wasted) {
                    pv.f(F::ACC, g) = acc;
                    pv.i(F::K, g) = k + 1;
                    stt = ST_DONE;
                } else {
#pragma unroll
                    for (int i = 0; i < D; ++i) { rec_x[i] = x[i]; rec_nin[i] = onN ? nin[i] : 0.f; rec_nu[i] = nu[i]; }
                    float xo[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) xo[i] = onN ? fmaf(G.tau, nin[i], x[i]) : x[i];
                    if (hp >= 0) {
                        // the walk's side of a Neumann primitive is the domain, so
                        // its normal toward the walk is -n_out (a first hit seen
                        // from inside is always an exit, nu . n_out > 0)
                        const float4 ex = G.neu.pextra[hp];
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            x[i] = fmaf(th, nu[i], xo[i]);
                            nin[i] = -(i == 0 ? ex.x : (i == 1 ? ex.y : ex.z));
                        }
                        onp = hp;
                    } else {
                        // the segment from the ray's origin to this point crosses
                        // no boundary, so the walker stays inside; stepping from
                        // x itself could leave the domain by up to tau along a
                        // grazing ray
#pragma unroll
                        for (int i = 0; i < D; ++i) x[i] = fmaf(r, nu[i], xo[i]);
                        onp = -1;
                    }
                    T *= w;
                    ++k;
                    stt = ST_ACTIVE;
                    // Russian roulette for the next star (played with that step's word)
                    if (k >= P.rr_start) {
                        const uint4 wr = walk_stream(P, wid).block((uint32_t)k, kBlkNeu);
                        if (u01(wr.w) >= P.rr_q) { stt = ST_DONE; ++n_rr; }
                        else T /= P.rr_q;
                    }
#pragma unroll
                    for (int i = 0; i < D; ++i) { pv.f(F::X + i, g) = x[i]; pv.f(F::NIN + i, g) = nin[i]; }
                    pv.i(F::ONP, g) = onp;
                    pv.f(F::T, g) = T;
                    pv.f(F::ACC, g) = acc;
                    pv.i(F::K, g) = k;
                    rec_pmis = pv.f(F::PMIS, g);
                    rec_prefix = acc;
                    rec_tnext = T;
                    do_rec = GUIDED && P.rec.data != nullptr;
                }
            }
            if (stt == ST_DONE) {
                if (!do_rec) wid = pv.wid(g);
                ++n_walks;
                P.slot_value[wid] = pv.f(F::ACC, g);
                if (P.slot_steps) P.slot_steps[wid] = pv.i(F::K, g);
                stt = ST_EMPTY;
            }
            // ---- training record append (one atomic per chunk)
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
                            dst[(int64_t)(3 * D + 3) * C] = __uint_as_float((uint32_t)wid);
                            dst[(int64_t)(3 * D + 4) * C] = 0.f;
                            ++n_rec;
                        } else {
                            ++n_drop;
                        }
                    }
                }
            }
            // ---- refill empty slots with new walks (wave-uniform control flow)
            if (!exhausted) {
                const uint64_t freem = __ballot(stt == ST_EMPTY);
                if (freem) {
                    const uint32_t cnt = (uint32_t)__popcll(freem);
                    if (pool_next >= pool_end) {
                        unsigned long long wb = 0;
                        if (lane == 0) wb = atomicAdd(P.work, (unsigned long long)P.chunk);
                        const uint32_t blo = __shfl((uint32_t)wb, 0), bhi = __shfl((uint32_t)(wb >> 32), 0);
                        wb = wave_uniform_u64(((unsigned long long)bhi << 32) | blo);
                        pool_next = wb;
                        pool_end = wb + P.chunk < P.n_walks ? wb + P.chunk : P.n_walks;
                        if (wb >= P.n_walks) exhausted = true;
                    }
                    const uint64_t avail = pool_end > pool_next ? pool_end - pool_next : 0;
                    if (stt == ST_EMPTY && !exhausted) {
                        const uint64_t rank = lane_prefix(freem);
                        if (rank < avail) {
                            const uint64_t id = pool_next + rank;
                            const uint64_t p = id / (uint64_t)P.wpp;
#pragma unroll
                            for (int i = 0; i < D; ++i) { pv.f(F::X + i, g) = P.pts[p * D + i]; pv.f(F::NIN + i, g) = 0.f; }
                            pv.i(F::ONP, g) = -1;
                            pv.f(F::T, g) = 1.f;
                            pv.f(F::ACC, g) = 0.f;
                            pv.f(F::DD, g) = 0.f;
                            pv.i(F::K, g) = 0;
                            pv.u(F::WLO, g) = (uint32_t)id;
                            pv.u(F::WHI, g) = (uint32_t)(id >> 32);
                            stt = ST_ACTIVE;
                        }
                    }
                    pool_next = wave_uniform_u64(pool_next + (cnt < avail ? cnt : avail));
                }
            }
            pv.i(F::STAT, g) = stt;
            const uint64_t am = __ballot(stt == ST_ACTIVE);
            if (stt == ST_ACTIVE) L_act[n_act + (int)lane_prefix(am)] = li;
            n_act += __popcll(am);
        }
        if (n_act == 0 && exhausted) break;
        // ---- once no new walks come, move the live walks to the front of
        // the pool whenever they fill at most half of the scanned prefix, so
        // that the last rounds scan a few chunks instead of the whole pool.
        // L_act is increasing, so a slot is only ever read by a list entry at
        // or before the one that overwrites it: within a chunk every lane's
        // load of a word returns before that word's store is issued, and
        // later chunks read slots beyond every earlier destination.  Walks
        // keep their ids and random streams, so every estimate is unchanged.
        if (exhausted && Nn > kWave && 2 * n_act <= Nn) {
            wave_sync();
            for (int r0 = 0; r0 < n_act; r0 += kWave) {
                const int r = r0 + lane;
                const int src = r < n_act ? L_act[r] : r;
                if (src != r) {
#pragma unroll 4
                    for (int f = 0; f < F::WORDS; ++f) {
                        const uint32_t v = pv.u(f, base + src);
                        pv.u(f, base + r) = v;
                    }
                }
            }
            const int n_new = (n_act + kWave - 1) / kWave * kWave;
            for (int r = n_act + lane; r < n_new; r += kWave) pv.i(F::STAT, base + r) = ST_EMPTY;
            wave_sync();
            for (int r = lane; r < n_act; r += kWave) L_act[r] = r;
            Nn = n_new;
        }
        wave_sync();
        // In 3D a closest-point query's length grows with the distance to the
        // Dirichlet boundary (the search ball), and the phase waits for its
        // longest query: list the walks whose last distance was at least the
        // mean first, so that those start early.  New walks count as short.
        if constexpr (D == 3) {
            list_long_first(L_act, Nn, base, lane, [&](uint32_t g) { return pv.i(F::STAT, g) == ST_ACTIVE; },
                            [&](uint32_t g) { return pv.f(F::DD, g); });
            wave_sync();
        }

        // ---- closest Dirichlet point; epsilon-shell and step-cap termination
        int n_step = 0;
        {
            float x[D];
            Trav q;
            run_phase(L_act, n_act, (int32_t*)nullptr, dummy_n, lane, batch, witer[0],
                [&](int slot) {
                    const uint32_t g = base + slot;
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
                    trav_begin(G.dir, INFINITY, q);
                },
                [&]() { return closest_dirichlet_step<D>(G.dir, x, q, st, &sq[0]); },
                [&](int slot) {
                    const uint32_t g = base + slot;
                    ++n_steps;
                    const float dD = q.prim >= 0 ? sqrtf(q.best) : INFINITY;
                    const int k = pv.i(F::K, g);
                    if (dD <= P.eps || k >= P.max_steps) {
                        float xbar[D];
                        float gv = 0.f;
                        if (q.prim >= 0) {
                            Prim<D> pr;
                            pr.load(G.dir.prims, q.prim);
                            pr.closest(x, xbar);
                            gv = field_value<D>(P.g, xbar);
                        }
                        pv.f(F::ACC, g) = fmaf(pv.f(F::T, g), gv, pv.f(F::ACC, g));
                        pv.i(F::K, g) = k + 1;
                        pv.i(F::STAT, g) = ST_DONE;
                        if (!(dD <= P.eps)) ++n_trunc;
                        return false;
                    }
                    pv.f(F::DD, g) = dD;
                    pv.i(F::STAT, g) = ST_STEP;
                    return true;
                });
        }
        wave_sync();
        // the walks that step on; the star's queries run longer far from the
        // Dirichlet boundary (a larger search radius) and on the Neumann
        // boundary, where normal cones prune less
        n_step = list_long_first(L_step, Nn, base, lane, [&](uint32_t g) { return pv.i(F::STAT, g) == ST_STEP; },
                                 [&](uint32_t g) { return pv.f(F::DD, g) * (pv.i(F::ONP, g) >= 0 ? 2.f : 1.f); });
        wave_sync();
        if (n_step == 0) continue;

        // ---- closest silhouette -> star radius; uniform direction
        {
            float x[D], dD = 0.f;
            int onp = -1, piece = -1;
            Trav q;
            run_phase(L_step, n_step, (int32_t*)nullptr, dummy_n, lane, batch, witer[1],
                [&](int slot) {
                    const uint32_t g = base + slot;
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
                    onp = pv.i(F::ONP, g);
                    dD = pv.f(F::DD, g);
                    piece = onp >= 0 && G.sil.piece ? G.sil.piece[onp] : -1;
                    trav_begin(G.sil, dD * dD, q);
                },
                [&]() { return closest_silhouette_step<D>(G.sil, x, onp, piece, q, st, &sq[1]); },
                [&](int slot) {
                    const uint32_t g = base + slot;
                    const float r = fmaxf(fminf(dD, sqrtf(q.best)), P.r_min);
                    pv.f(F::R, g) = r;
                    pv.f(F::CON, g) = 0.f;
                    if constexpr (!GUIDED) {
                        const Stream rs = walk_stream(P, pv.wid(g));
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
                    return false;
                });
        }
        wave_sync();

        // ---- guided direction: the network for 64 walks at a time on MFMA,
        // then each lane draws from its own mixture
        if constexpr (GUIDED) {
            for (int c0 = 0; c0 < n_step; c0 += kWave) {
                const int idx = c0 + lane;
                const bool valid = idx < n_step;
                const uint32_t g = base + L_step[valid ? idx : c0];
                float x[D];
#pragma unroll
                for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
                __syncthreads();
                guide_forward_wave<D>(P.guide, x, s_out, lane, out_stride);
                __syncthreads();
                if (valid) {
                    const int onp = pv.i(F::ONP, g);
                    const bool onN = onp >= 0;
                    float nin[D], nu[D], pmis = 1.f / area;
#pragma unroll
                    for (int i = 0; i < D; ++i) nin[i] = pv.f(F::NIN + i, g);
                    const int k = pv.i(F::K, g);
                    const Stream rs = walk_stream(P, pv.wid(g));
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
            wave_sync();
        }

        // ---- Neumann contribution: area-weighted point on a Neumann
        // primitive meeting the ball, kept if it lies in the star
        if (has_h) {
            int n_vis = 0;
            {
                float x[D], r = 0.f, u1 = 0.f, u2 = 0.f;
                SampleTrav q;
                run_phase(L_step, n_step, L_vis, n_vis, lane, batch, witer[2],
                    [&](int slot) {
                        const uint32_t g = base + slot;
#pragma unroll
                        for (int i = 0; i < D; ++i) x[i] = pv.f(F::X + i, g);
                        r = pv.f(F::R, g);
                        const uint4 wn = walk_stream(P, pv.wid(g)).block((uint32_t)pv.i(F::K, g), kBlkNeu);
                        u1 = u01(wn.y);
                        u2 = u01(wn.z);
                        sample_begin(G.neu, u01(wn.x), q);
                    },
                    [&]() { return sample_neumann_step<D>(G.neu, x, r, q, &sq[2]); },
                    [&](int slot) {
                        if (!(q.prim >= 0 && q.prob > 0.f)) return false;
                        const uint32_t g = base + slot;
                        Prim<D> pr;
                        pr.load(G.neu.prims, q.prim);
                        float z[D], dz[D], rho2 = 0.f;
                        pr.point(u1, u2, z);
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
                        if (!ok) return false;
                        const float4 ex = G.neu.pextra[q.prim];
                        const float no[3] = {ex.x, ex.y, ex.z};
                        const float hv = neumann_value<D>(P.h, z, no);
                        const float inv_alpha = onp >= 0 ? 2.f : 1.f;
                        pv.f(F::NVAL, g) = green_ball<D>(r, rho) * hv * (ex.w / q.prob) * inv_alpha;
#pragma unroll
                        for (int i = 0; i < D; ++i) pv.f(F::Z + i, g) = z[i];
                        // the sample's primitive, for its visibility ray (the
                        // hit field is free until the first-hit phase)
                        pv.i(F::HIT, g) = q.prim;
                        return true;
                    });
            }
            wave_sync();
            if (n_vis > 0) {
                float xo[D], dn[D];
                int onp = -1, zp = -1;
                RayTrav<D> q;
                run_phase(L_vis, n_vis, (int32_t*)nullptr, dummy_n, lane, batch, witer[3],
                    [&](int slot) {
                        const uint32_t g = base + slot;
                        onp = pv.i(F::ONP, g);
                        zp = pv.i(F::HIT, g);
                        float l2 = 0.f;
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
                        ray_begin<D>(G.neu, dn, len - G.tau, q);
                    },
                    [&]() { return visible_neumann_step<D>(G.neu, xo, dn, 0.f, onp, zp, q, st, &sq[3]); },
                    [&](int slot) {
                        const uint32_t g = base + slot;
                        if (q.t.prim < 0) pv.f(F::CON, g) += pv.f(F::NVAL, g);
                        return false;
                    });
                wave_sync();
            }
        }

        // ---- source contribution: radius from the radial law of the ball's
        // Green's function, uniform direction, kept if visible in the star
        if (has_f) {
            int n_svis = 0;
            for (int c0 = 0; c0 < n_step; c0 += kWave) {
                const int idx = c0 + lane;
                bool app = false;
                int slot = -1;
                if (idx < n_step) {
                    slot = L_step[idx];
                    const uint32_t g = base + slot;
                    const Stream rs = walk_stream(P, pv.wid(g));
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
                const uint64_t m = __ballot(app);
                if (m) {
                    if (app) L_svis[n_svis + (int)lane_prefix(m)] = slot;
                    n_svis += __popcll(m);
                }
            }
            wave_sync();
            if (n_svis > 0) {
                float xo[D], dy[D];
                int onp = -1;
                RayTrav<D> q;
                run_phase(L_svis, n_svis, (int32_t*)nullptr, dummy_n, lane, batch, witer[4],
                    [&](int slot) {
                        const uint32_t g = base + slot;
                        onp = pv.i(F::ONP, g);
                        float l2 = 0.f;
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
                        ray_begin<D>(G.neu, dy, len, q);
                    },
                    [&]() { return visible_neumann_step<D>(G.neu, xo, dy, 0.f, onp, -1, q, st, &sq[4]); },
                    [&](int slot) {
                        if (q.t.prim < 0) {
                            const uint32_t g = base + slot;
                            pv.f(F::CON, g) -= pv.f(F::SVAL, g);
                        }
                        return false;
                    });
                wave_sync();
            }
        }

        // ---- first hit inside the star
        {
            float xo[D], nu[D];
            int onp = -1;
            RayTrav<D> q;
            run_phase(L_step, n_step, (int32_t*)nullptr, dummy_n, lane, batch, witer[5],
                [&](int slot) {
                    const uint32_t g = base + slot;
                    onp = pv.i(F::ONP, g);
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        const float xi = pv.f(F::X + i, g);
                        xo[i] = onp >= 0 ? fmaf(G.tau, pv.f(F::NIN + i, g), xi) : xi;
                        nu[i] = pv.f(F::NU + i, g);
                    }
                    // the search runs to r + tau, so a boundary point at
                    // distance r (a silhouette point straight ahead) puts the
                    // walker on the boundary, and exits up to tau behind the
                    // origin count (the origin is then on the boundary up to
                    // rounding)
                    ray_begin<D>(G.neu, nu, pv.f(F::R, g) + G.tau, q);
                },
                [&]() { return ray_neumann_step<D>(G.neu, xo, nu, 0.f, G.tau, onp, q, st, &sq[5]); },
                [&](int slot) {
                    const uint32_t g = base + slot;
                    pv.f(F::TH, g) = q.t.prim >= 0 ? q.t.best : INFINITY;
                    pv.i(F::HIT, g) = q.t.prim;
                    return false;
                });
        }
        wave_sync();
    }

    // ---- statistics: one atomic per wave and counter
    if constexpr (STATS) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const unsigned long long a = wave_sum_u64(sq[q].nodes), b = wave_sum_u64(sq[q].prims);
            if (lane == 0) {
                atomicAdd(P.cost + 2 * q, a);
                atomicAdd(P.cost + 2 * q + 1, b);
                atomicAdd(P.cost + 12 + q, witer[q]);
            }
        }
    }
    const uint32_t vals[7] = {n_steps, n_walks, n_trunc, n_rr, n_bad, n_rec, n_drop};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const unsigned long long sm = wave_sum_u64(vals[i]);
        if (lane == 0 && sm) atomicAdd(P.counters + i, sm);
    }
}

// Register bounds per variant (resident waves per SIMD); the traversal
// phases are latency-bound, so residency matters more than a few spills of
// values that live across phases.
#ifndef WOST_WAVES_2D_UNIFORM
#define WOST_WAVES_2D_UNIFORM 5
#endif
#ifndef WOST_WAVES_2D_GUIDED
#define WOST_WAVES_2D_GUIDED 4
#endif
template <bool STATS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WOST_WAVES_2D_UNIFORM))) void walk_kernel2u(const WalkParams P)
{
    walk_body<2, false, STATS>(P);
}

template <bool STATS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WOST_WAVES_2D_GUIDED))) void walk_kernel2g(const WalkParams P)
{
    walk_body<2, true, STATS>(P);
}

#ifndef WOST_WAVES_3D_UNIFORM
#define WOST_WAVES_3D_UNIFORM 3
#endif
#ifndef WOST_WAVES_3D_GUIDED
#define WOST_WAVES_3D_GUIDED 3
#endif
template <bool STATS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WOST_WAVES_3D_UNIFORM))) void walk_kernel3u(const WalkParams P)
{
    walk_body<3, false, STATS>(P);
}

template <bool STATS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WOST_WAVES_3D_GUIDED))) void walk_kernel3g(const WalkParams P)
{
    walk_body<3, true, STATS>(P);
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
__global__ __launch_bounds__(64) void query_kernel(const DevGeom G, const float* pts, int64_t n, const int32_t* on_prim,
                                                   float* d_dir,
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
    if (d_sil) {
        // a point on a Neumann primitive sees that primitive from the front
        const int32_t q = on_prim ? on_prim[i] : -1;
        const int onp = q >= 0 && q < G.n_caller && G.neu_id ? G.neu_id[q] : -1;
        d_sil[i] = sqrtf(closest_silhouette<D>(G.sil, x, INFINITY, onp, st));
    }
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

// The walk's Neumann-sample step for given states (for parity tests): the
// descent choosing one primitive meeting B(x, r), the point on it, the
// in-ball and facing checks, and the visibility ray from the walker's origin
// -- the same steps, in the same order and precision, as the Neumann phase of
// walk_body.
template <int D>
__global__ __launch_bounds__(64) void neumann_sample_kernel(const DevGeom G, const float* pts, int64_t n,
                                                            const int32_t* on_prim, const float* radius,
                                                            const float* uni, int32_t* prim_out, float* prob_out,
                                                            float* z_out, int32_t* ok_out)
{
    __shared__ uint2 s_stack[kMaxStack * kWave];
    const int lane = threadIdx.x;
    const LdsStack st{&s_stack[lane]};
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    if (i >= n) return;
    float x[D], nin[D];
#pragma unroll
    for (int c = 0; c < D; ++c) { x[c] = pts[i * D + c]; nin[c] = 0.f; }
    const int32_t qc = on_prim ? on_prim[i] : -1;
    const int onp = qc >= 0 && qc < G.n_caller && G.neu_id ? G.neu_id[qc] : -1;
    if (onp >= 0) {
        const float4 ex = G.neu.pextra[onp];
#pragma unroll
        for (int c = 0; c < D; ++c) nin[c] = -(c == 0 ? ex.x : (c == 1 ? ex.y : ex.z));
    }
    const float r = radius[i];
    SampleTrav q;
    sample_begin(G.neu, uni[i * 3], q);
    while (!sample_neumann_step<D>(G.neu, x, r, q, (NoStat*)nullptr)) {}
    prim_out[i] = q.prim >= 0 ? G.neu.orig[q.prim] : -1;
    prob_out[i] = q.prob;
    int ok = 0;
    float z[D];
#pragma unroll
    for (int c = 0; c < D; ++c) z[c] = INFINITY;
    if (q.prim >= 0 && q.prob > 0.f) {
        Prim<D> pr;
        pr.load(G.neu.prims, q.prim);
        float dz[D], rho2 = 0.f;
        pr.point(uni[i * 3 + 1], uni[i * 3 + 2], z);
#pragma unroll
        for (int c = 0; c < D; ++c) { dz[c] = z[c] - x[c]; rho2 = fmaf(dz[c], dz[c], rho2); }
        const float rho = sqrtf(rho2);
        bool acc = rho < r && rho > 0.f;
        if (acc && onp >= 0 && dot<D>(dz, nin) < -G.tau) acc = false;
        if (acc) {
            float xo[D], dn[D], l2 = 0.f;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                xo[c] = onp >= 0 ? fmaf(G.tau, nin[c], x[c]) : x[c];
                dn[c] = z[c] - xo[c];
                l2 = fmaf(dn[c], dn[c], l2);
            }
            const float len = sqrtf(l2);
#pragma unroll
            for (int c = 0; c < D; ++c) dn[c] /= len;
            RayTrav<D> rq;
            ray_begin<D>(G.neu, dn, len - G.tau, rq);
            while (!visible_neumann_step<D>(G.neu, xo, dn, 0.f, onp, q.prim, rq, st, (NoStat*)nullptr)) {}
            ok = rq.t.prim < 0 ? 1 : 0;
        }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) z_out[i * D + c] = z[c];
    ok_out[i] = ok;
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

// Walk slots per wave, default per dimension (2D, 3D): larger pools give each
// phase more walks to hand out, which hides more of the fetch latency of the
// 3D queries (measured: 2D best at 384, 3D at 1536 -- 1.2-1.4x over 384)
constexpr int kDefaultPoolSlots[2] = {384, 1536};
static int g_pool_n = 0;   // 0: the default of the solve's dimension
static inline int pool_n_of(int dim) { return g_pool_n ? g_pool_n : kDefaultPoolSlots[dim == 3]; }
static inline int refill_of(int dim) { return g_refill_batch ? g_refill_batch : kDefaultRefillBatch[dim == 3]; }
#ifndef WOST_POOL_MIN
#define WOST_POOL_MIN 64
#endif
static int g_pool_min = WOST_POOL_MIN;   // fewest walks per wave before the grid shrinks

static inline int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }
static inline int pool_words(int dim) { return dim == 2 ? PoolField<2>::WORDS : PoolField<3>::WORDS; }

// Slots per wave for a launch of `grid` waves: enough to hold the launch's
// walks at once, at most the pool size, a multiple of 64.
static inline int pool_slots(uint64_t n_walks, int grid, int dim)
{
    const uint64_t per = (n_walks + (uint64_t)grid - 1) / (uint64_t)grid;
    const uint64_t n64 = (per + 63) / 64 * 64;
    return (int)std::max<uint64_t>(64, std::min<uint64_t>(n64, (uint64_t)pool_n_of(dim)));
}

// Upper bound of the pool slots of any launch (grid <= 32 waves per CU and
// grid <= ceil(walks / 64)): grid * pool_slots <= walks + 64 grid + 64.
static inline int64_t pool_slots_bound(uint64_t n_walks, int dim)
{
    const uint64_t cap = (uint64_t)num_cu() * 32;
    const uint64_t gmax = std::min<uint64_t>(cap, (n_walks + 63) / 64);
    return (int64_t)std::min<uint64_t>(cap * (uint64_t)pool_n_of(dim), n_walks + 64 * gmax + 64);
}

extern "C" int64_t wost_solve_workspace_bytes(const wost_geom* geom, int64_t n_points, int32_t wpp)
{
    if (!geom || n_points < 0 || wpp <= 0) return -1;
    const uint64_t n_walks = (uint64_t)n_points * (uint64_t)wpp;
    const int64_t slots = pool_slots_bound(n_walks, geom->dim);
    return 256 + align256((int64_t)n_walks * 4) + align256(slots * pool_words(geom->dim) * 4) + align256(slots * 4 * 4);
}

extern "C" int wost_set_walk_pool(int32_t slots_per_wave, int32_t refill_batch)
{
    if (slots_per_wave != 0 && (slots_per_wave < 64 || slots_per_wave > 8192 || slots_per_wave % 64)) {
        set_error("wost_set_walk_pool: slots_per_wave must be a multiple of 64 in [64, 8192] (0 = default)");
        return WOST_EINVAL;
    }
    if (refill_batch != 0 && (refill_batch < 1 || refill_batch > 64)) {
        set_error("wost_set_walk_pool: refill_batch must be in [1, 64] (0 = default)");
        return WOST_EINVAL;
    }
    g_pool_n = slots_per_wave;
    g_refill_batch = refill_batch;
    return WOST_OK;
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

namespace wost {

// Checks a solve's arguments and fills the launch parameters both solvers
// share (geometry, fields, problem, random streams, guide, records, output
// buffers); `who` names the entry point in error messages.
int prepare_solve(const char* who, const wost_geom* geom, const wost_problem* pb, const float* pts, int64_t n_points,
                  int32_t wpp, uint64_t seed, uint64_t walk_offset, const wost_guide* guide, double* sum,
                  double* sum_sq, int64_t* count, float* walk_value, int32_t* walk_steps, const wost_records* rec,
                  void* workspace, uint64_t* dev_counters, WalkParams& P)
{
    if (!geom || !pb || !pts || !sum || !sum_sq || !count || !workspace || !dev_counters) {
        set_error("%s: NULL argument", who);
        return WOST_EINVAL;
    }
    if (!geom->dev) { set_error("%s: geometry not uploaded", who); return WOST_ESTATE; }
    if (geom->n_dir == 0) { set_error("%s: the boundary has no Dirichlet part (walks never end)", who); return WOST_EINVAL; }
    if (n_points <= 0 || wpp <= 0) { set_error("%s: n_points and wpp must be positive", who); return WOST_EINVAL; }
    if (n_points > 0xFFFFFFFFll || walk_offset + (uint64_t)wpp > 0xFFFFFFFFull) {
        set_error("%s: point index and walk index must fit 32 bits", who);
        return WOST_EUNSUPPORTED;
    }
    if (!(pb->eps > 0.f) || pb->max_steps < 0 || !(pb->rr_q > 0.f && pb->rr_q <= 1.f) || pb->r_min < 0.f) {
        set_error("%s: need eps > 0, max_steps >= 0, 0 < rr_q <= 1, r_min >= 0", who);
        return WOST_EINVAL;
    }
    const bool guided = pb->sampling != WOST_SAMPLING_UNIFORM;
    if (pb->sampling < 0 || pb->sampling > WOST_SAMPLING_GUIDED_ONLY) { set_error("%s: unknown sampling mode", who); return WOST_EINVAL; }
    if (guided != (guide != nullptr)) { set_error("%s: guide must be given iff sampling is not UNIFORM", who); return WOST_EINVAL; }
    if (pb->sampling == WOST_SAMPLING_MIS_FIXED && !(pb->c_fixed >= 0.f && pb->c_fixed <= 1.f)) {
        set_error("%s: c_fixed must be in [0, 1]", who);
        return WOST_EINVAL;
    }
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
    if (guided && guide && (pb->reflect != 0) != (guide->dev.reflect != 0)) {
        // the training loss reads the guide's setting, so a solve that draws
        // otherwise would train against another density than it sampled
        set_error("%s: problem.reflect = %d but the guide's reflection setting is %d "
                  "(wost_guide_set_reflect)", who, pb->reflect != 0, guide->dev.reflect != 0);
        return WOST_EINVAL;
    }
    if (guided) {
        int rc = guide_prepare(guide, dim, P.guide);
        if (rc != WOST_OK) return rc;
        P.guide.sampling = pb->sampling;
        P.guide.c_fixed = pb->c_fixed;
        P.guide.reflect = pb->reflect != 0;
    }
    if (rec) {
        if (!guided) { set_error("%s: training records need a guided sampling mode", who); return WOST_EINVAL; }
        if (!rec->data || !rec->count || rec->capacity < 0) { set_error("%s: bad record buffer", who); return WOST_EINVAL; }
        P.rec.data = rec->data;
        P.rec.capacity = rec->capacity;
        P.rec.count = (unsigned long long*)rec->count;
    }
    return WOST_OK;
}

int walk_num_cu() { return num_cu(); }

void launch_reduce_points(const WalkParams& P, double* sum, double* sum_sq, int64_t* count, hipStream_t s)
{
    const int rgrid = (int)((P.n_points + 3) / 4);
    hipLaunchKernelGGL(reduce_points, dim3(rgrid), dim3(256), 0, s, P.slot_value, P.n_points, P.wpp, sum, sum_sq,
                       count);
}

}  // namespace wost

extern "C" int wost_solve(const wost_geom* geom, const wost_problem* pb, const float* pts, int64_t n_points,
                          int32_t wpp, uint64_t seed, uint64_t walk_offset, const wost_guide* guide, double* sum,
                          double* sum_sq, int64_t* count, float* walk_value, int32_t* walk_steps,
                          const wost_records* rec, void* workspace, int64_t ws_bytes, uint64_t* dev_counters,
                          void* stream)
{
    WalkParams P;
    int rc = prepare_solve("wost_solve", geom, pb, pts, n_points, wpp, seed, walk_offset, guide, sum, sum_sq, count,
                           walk_value, walk_steps, rec, workspace, dev_counters, P);
    if (rc != WOST_OK) return rc;
    const int64_t need = wost_solve_workspace_bytes(geom, n_points, wpp);
    if (ws_bytes < need) { set_error("wost_solve: workspace %lld < %lld bytes", (long long)ws_bytes, (long long)need); return WOST_ESIZE; }
    const bool guided = pb->sampling != WOST_SAMPLING_UNIFORM;
    const int dim = geom->dim;
    uint8_t* ws = (uint8_t*)workspace;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, P.work, 1);
    using WalkFn = void (*)(const WalkParams);
    WalkFn fn;
    if (dim == 2) {
        if (P.cost) fn = guided ? walk_kernel2g<true> : walk_kernel2u<true>;
        else fn = guided ? walk_kernel2g<false> : walk_kernel2u<false>;
    } else {
        if (P.cost) fn = guided ? walk_kernel3g<true> : walk_kernel3u<true>;
        else fn = guided ? walk_kernel3g<false> : walk_kernel3u<false>;
    }
    const size_t lds = walk_lds_bytes(guided, geom->stack_need(), guide_out_stride(P.guide));
    int per_cu = g_waves_per_cu;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, lds) != hipSuccess || nb < 1) nb = 8;
        per_cu = nb;
    }
    const uint64_t waves_needed = (P.n_walks + 63) / 64;
    const uint64_t cap = (uint64_t)num_cu() * (uint64_t)std::min(per_cu, 32);
    // fewer, fuller waves for launches that would leave pools short: each
    // wave gets at least g_pool_min walks while the chip keeps at least
    // 4 waves per CU
    uint64_t want = waves_needed;
    if (g_pool_min > 64) want = std::max<uint64_t>((uint64_t)num_cu() * 4, (P.n_walks + g_pool_min - 1) / g_pool_min);
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(std::min<uint64_t>(waves_needed, want), cap));
    P.pool_n = pool_slots(P.n_walks, grid, dim);
    P.refill_batch = refill_of(dim);
    P.pool_total = (int64_t)grid * P.pool_n;
    {
        // workspace: counter | per-walk values | pools | work lists
        const int64_t vbytes = align256((int64_t)P.n_walks * 4);
        const int64_t pbytes = align256(P.pool_total * pool_words(dim) * 4);
        if ((uint64_t)P.pool_total * (uint64_t)pool_words(dim) >= (1ull << 32)) {
            set_error("wost_solve: walk pools exceed 2^32 words; lower wost_set_walk_pool");
            return WOST_EUNSUPPORTED;
        }
        if (P.pool_total > pool_slots_bound(P.n_walks, dim) || 256 + vbytes + pbytes + align256(P.pool_total * 16) > ws_bytes) {
            set_error("wost_solve: workspace too small for the launch");
            return WOST_ESIZE;
        }
        P.pool = (uint32_t*)(ws + 256 + vbytes);
        P.lists = (int32_t*)(ws + 256 + vbytes + pbytes);
    }
    // about eight reservations per wave over the whole call, at least one lane's worth each
    P.chunk = std::max<uint64_t>(64, std::min<uint64_t>(4096, P.n_walks / ((uint64_t)grid * 8)));
    hipLaunchKernelGGL(fn, dim3(grid), dim3(64), lds, s, P);
    launch_reduce_points(P, sum, sum_sq, count, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_solve: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_neumann_sample(const wost_geom* geom, const float* pts, int64_t n, const int32_t* on_prim,
                                   const float* radius, const float* uniforms, int32_t* prim, float* prob, float* z,
                                   int32_t* accepted, void* stream)
{
    if (!geom) { set_error("wost_neumann_sample: NULL geometry"); return WOST_EINVAL; }
    if (!geom->dev) { set_error("wost_neumann_sample: geometry not uploaded"); return WOST_ESTATE; }
    if (n < 0) { set_error("wost_neumann_sample: n < 0"); return WOST_EINVAL; }
    if (n == 0) return WOST_OK;
    if (!pts || !radius || !uniforms || !prim || !prob || !z || !accepted) {
        set_error("wost_neumann_sample: NULL buffer");
        return WOST_EINVAL;
    }
    const DevGeom G = geom->devgeom();
    hipStream_t s = (hipStream_t)stream;
    const int grid = (int)((n + 63) / 64);
    if (geom->dim == 2)
        hipLaunchKernelGGL(neumann_sample_kernel<2>, dim3(grid), dim3(64), 0, s, G, pts, n, on_prim, radius, uniforms,
                           prim, prob, z, accepted);
    else
        hipLaunchKernelGGL(neumann_sample_kernel<3>, dim3(grid), dim3(64), 0, s, G, pts, n, on_prim, radius, uniforms,
                           prim, prob, z, accepted);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_neumann_sample: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_query(const wost_geom* geom, const float* pts, int64_t n, const int32_t* on_prim, float* d_dir,
                          float* xbar, float* d_sil, const float* ray_dir, const float* ray_tmax, float* ray_t,
                          int32_t* ray_prim, void* stream)
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
        hipLaunchKernelGGL(query_kernel<2>, dim3(grid), dim3(64), 0, s, G, pts, n, on_prim, d_dir, xbar, d_sil, ray_dir,
                           ray_tmax, ray_t, ray_prim);
    else
        hipLaunchKernelGGL(query_kernel<3>, dim3(grid), dim3(64), 0, s, G, pts, n, on_prim, d_dir, xbar, d_sil, ray_dir,
                           ray_tmax, ray_t, ray_prim);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_query: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}
