// Device-side boundary queries of one walk step (gfx950, FP32).
//
//  closest_dirichlet  distance / closest point to the Dirichlet boundary
//                     (epsilon-shell test and terminal value, Sec. 3.2)
//  closest_silhouette distance to the nearest Neumann silhouette point seen
//                     from x (bounds the star radius, Sec. 3.2); normal cones
//                     prune subtrees whose primitives all face x the same way
//  ray_neumann        first Neumann hit in (tau, tmax): next walk location
//  visible_neumann    no Neumann primitive crosses the open segment (x, z)
//  sample_neumann     one area-weighted primitive among those meeting the ball,
//                     by a single descent with subtree measures as weights
//
// Every traversal keeps its stack in LDS: column `lane` of a
// [kMaxStack][64] array of (node, key) pairs; consecutive lanes hit
// consecutive banks.
#pragma once

#include "wost_internal.h"

namespace wost {

struct LdsStack {
    uint2* base;    // &stack[0][lane]
    __device__ __forceinline__ void put(int i, int node, float key) const
    {
        base[i * kWave] = make_uint2((uint32_t)node, __float_as_uint(key));
    }
    __device__ __forceinline__ uint2 get(int i) const { return base[i * kWave]; }
};

template <int D> struct Box { float lo[D], hi[D]; };

// Traversal cost counters: NoStat compiles to nothing; Stat counts node
// fetches and primitive tests of one query type.
struct NoStat {};
struct Stat {
    uint32_t nodes = 0, prims = 0;
    uint32_t step0 = 0;             // nodes at the start of the current walk step
    unsigned long long witer = 0;   // wave-level iterations (lane 0 only)
};
__device__ __forceinline__ void stat_node(NoStat*) {}
__device__ __forceinline__ void stat_prim(NoStat*) {}
__device__ __forceinline__ void stat_node(Stat* s) { ++s->nodes; }
__device__ __forceinline__ void stat_prim(Stat* s) { ++s->prims; }

// component k of a float4 / int4 (k is a compile-time constant after unrolling)
__device__ __forceinline__ float comp(const float4& v, int k)
{
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}
__device__ __forceinline__ int comp(const int4& v, int k)
{
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// The four children's boxes and references of one four-wide node.
template <int D> struct Node4 {
    float4 lo[D], hi[D];
    int4 ref;
    __device__ __forceinline__ Box<D> box(int k) const
    {
        Box<D> b;
#pragma unroll
        for (int a = 0; a < D; ++a) { b.lo[a] = comp(lo[a], k); b.hi[a] = comp(hi[a], k); }
        return b;
    }
};

template <int D>
__device__ __forceinline__ const float4* node_ptr(const float4* nodes, int i, int stride)
{
    return nodes + (size_t)i * (size_t)stride;
}

template <int D>
__device__ __forceinline__ void load_node4(const float4* p, Node4<D>& n)
{
#pragma unroll
    for (int a = 0; a < D; ++a) { n.lo[a] = p[a]; n.hi[a] = p[D + a]; }
    const float4 r = p[2 * D];
    n.ref = make_int4(__float_as_int(r.x), __float_as_int(r.y), __float_as_int(r.z), __float_as_int(r.w));
}

template <int D>
__device__ __forceinline__ float box_dist2(const Box<D>& b, const float* x)
{
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float t = fmaxf(fmaxf(b.lo[i] - x[i], x[i] - b.hi[i]), 0.f);
        s = fmaf(t, t, s);
    }
    return s;
}

template <int D>
__device__ __forceinline__ float dot(const float* a, const float* b)
{
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) s = fmaf(a[i], b[i], s);
    return s;
}

// ----------------------------------------------------------------- primitives

// closest point on segment [a, a + e]; returns squared distance
template <int D>
__device__ __forceinline__ float closest_seg(const float* x, const float* a, const float* e, float* out)
{
    float w[D];
#pragma unroll
    for (int i = 0; i < D; ++i) w[i] = x[i] - a[i];
    const float ee = dot<D>(e, e);
    // parameter of the projection, clamped to the segment; the hardware
    // reciprocal (1 ulp) is enough for a value that is clamped and only
    // places the closest point
    float t = ee > 0.f ? dot<D>(w, e) * __builtin_amdgcn_rcpf(ee) : 0.f;
    t = fminf(fmaxf(t, 0.f), 1.f);
    float d2 = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        out[i] = fmaf(t, e[i], a[i]);
        const float u = x[i] - out[i];
        d2 = fmaf(u, u, d2);
    }
    return d2;
}

// closest point on triangle (a, a+ab, a+ac) by Voronoi-region classification
// (Ericson, Real-Time Collision Detection, Sec. 5.1.5); squared distance
__device__ __forceinline__ float closest_tri(const float* x, const float* a, const float* ab, const float* ac,
                                             float* out)
{
    float ap[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
    const float d1 = dot<3>(ab, ap), d2 = dot<3>(ac, ap);
    float u = 0.f, v = 0.f;   // out = a + u ab + v ac
    bool done = false;
    if (d1 <= 0.f && d2 <= 0.f) { done = true; }
    float bp[3] = {ap[0] - ab[0], ap[1] - ab[1], ap[2] - ab[2]};
    const float d3 = dot<3>(ab, bp), d4 = dot<3>(ac, bp);
    if (!done && d3 >= 0.f && d4 <= d3) { u = 1.f; done = true; }
    const float vc = d1 * d4 - d3 * d2;
    if (!done && vc <= 0.f && d1 >= 0.f && d3 <= 0.f) { u = d1 / (d1 - d3); done = true; }
    float cp[3] = {ap[0] - ac[0], ap[1] - ac[1], ap[2] - ac[2]};
    const float d5 = dot<3>(ab, cp), d6 = dot<3>(ac, cp);
    if (!done && d6 >= 0.f && d5 <= d6) { v = 1.f; done = true; }
    const float vb = d5 * d2 - d1 * d6;
    if (!done && vb <= 0.f && d2 >= 0.f && d6 <= 0.f) { v = d2 / (d2 - d6); done = true; }
    const float va = d3 * d6 - d5 * d4;
    if (!done && va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) {
        const float w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        u = 1.f - w; v = w; done = true;
    }
    if (!done) {
        const float den = 1.f / (va + vb + vc);
        u = vb * den; v = vc * den;
    }
    float d2s = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out[i] = a[i] + u * ab[i] + v * ac[i];
        const float t = x[i] - out[i];
        d2s = fmaf(t, t, d2s);
    }
    return d2s;
}

// Per-ray constants of the primitive hit tests.  Both tests are watertight:
// a ray crossing the boundary where primitives meet (a shared vertex in 2D, a
// shared edge in 3D) hits at least one of them, so a walker can never slip
// out of the domain between two primitives.
template <int D> struct RaySetup;
template <> struct RaySetup<2> {
    float x[2], nu[2];
    __device__ __forceinline__ RaySetup(const float* o, const float* d)
    {
        x[0] = o[0]; x[1] = o[1]; nu[0] = d[0]; nu[1] = d[1];
    }
    // side of vertex v relative to the ray's line: nu x (v - x).  A function of
    // (x, nu, v) alone, evaluated without contraction, so both segments that
    // share v see the same value there.
    __device__ __forceinline__ float side(float vx, float vy) const
    {
#pragma clang fp contract(off)
        return nu[0] * (vy - x[1]) - nu[1] * (vx - x[0]);
    }
};
// 3D: shear the ray onto +z (Woop, Benthin and Wald, "Watertight Ray/Triangle
// Intersection", JCGT 2013).  The shear is kept as three row vectors so a
// vertex maps to (px.v, py.v, pz.v) with no component permutation at run time;
// the products with 0 and 1 in those rows are exact, so each sheared coordinate
// is the same single rounding the permuted formulation would give.  These
// regions switch floating-point contraction off: a fused multiply-add would
// round the two products of an edge function differently in the two
// triangles that share the edge.
template <> struct RaySetup<3> {
    float x[3], px[3], py[3], pz[3];
    __device__ __forceinline__ RaySetup(const float* o, const float* d)
    {
        const float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
        const int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
        int kx = kz == 2 ? 0 : kz + 1, ky = kx == 2 ? 0 : kx + 1;
        const float dz = kz == 0 ? d[0] : (kz == 1 ? d[1] : d[2]);
        if (dz < 0.f) { const int t = kx; kx = ky; ky = t; }
        const float dx = kx == 0 ? d[0] : (kx == 1 ? d[1] : d[2]);
        const float dy = ky == 0 ? d[0] : (ky == 1 ? d[1] : d[2]);
        const float sx = dx / dz, sy = dy / dz, sz = 1.f / dz;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] = o[i];
            px[i] = (i == kx ? 1.f : 0.f) - (i == kz ? sx : 0.f);
            py[i] = (i == ky ? 1.f : 0.f) - (i == kz ? sy : 0.f);
            pz[i] = i == kz ? sz : 0.f;
        }
    }
    __device__ __forceinline__ void shear(const float* v, float& X, float& Y, float& Z) const
    {
#pragma clang fp contract(off)
        const float a0 = v[0] - x[0], a1 = v[1] - x[1], a2 = v[2] - x[2];
        X = (px[0] * a0 + px[1] * a1) + px[2] * a2;
        Y = (py[0] * a0 + py[1] * a1) + py[2] * a2;
        Z = (pz[0] * a0 + pz[1] * a1) + pz[2] * a2;
    }
};

// primitives of a leaf fetched together before they are tested
constexpr int kPrimGroup = 4;

template <int D> struct Prim;
// 2D segment from one float4 (a, b)
template <> struct Prim<2> {
    float a[2], b[2], e[2];
    __device__ __forceinline__ void load(const float4* p, int i)
    {
        const float4 s = p[i];
        a[0] = s.x; a[1] = s.y; b[0] = s.z; b[1] = s.w;
        e[0] = s.z - s.x; e[1] = s.w - s.y;
    }
    __device__ __forceinline__ float closest(const float* x, float* out) const { return closest_seg<2>(x, a, e, out); }
    // ray x + t nu against the closed segment; returns t or +inf.  The line
    // meets the segment iff its endpoints are not strictly on one side (a
    // segment lying on the line counts as missed).
    __device__ __forceinline__ float ray(const RaySetup<2>& r) const
    {
        const float oa = r.side(a[0], a[1]), ob = r.side(b[0], b[1]);
        if ((oa > 0.f && ob > 0.f) || (oa < 0.f && ob < 0.f) || (oa == 0.f && ob == 0.f)) return INFINITY;
        // crossing point a + s e; the hit decision above is exact, the
        // parameter only places the point (hardware reciprocal, clamped)
        const float s = fminf(fmaxf(oa * __builtin_amdgcn_rcpf(oa - ob), 0.f), 1.f);
        const float cx = fmaf(s, e[0], a[0]) - r.x[0], cy = fmaf(s, e[1], a[1]) - r.x[1];
        return fmaf(cx, r.nu[0], cy * r.nu[1]);
    }
    __device__ __forceinline__ void point(float s, float, float* z) const
    {
        z[0] = fmaf(s, e[0], a[0]);
        z[1] = fmaf(s, e[1], a[1]);
    }
};
// 3D triangle from three float4 (a, b, c)
template <> struct Prim<3> {
    float a[3], b[3], c[3], e1[3], e2[3];
    __device__ __forceinline__ void load(const float4* p, int i)
    {
        const float4 s0 = p[3 * i], s1 = p[3 * i + 1], s2 = p[3 * i + 2];
        a[0] = s0.x; a[1] = s0.y; a[2] = s0.z;
        b[0] = s0.w; b[1] = s1.x; b[2] = s1.y;
        c[0] = s1.z; c[1] = s1.w; c[2] = s2.x;
#pragma unroll
        for (int k = 0; k < 3; ++k) { e1[k] = b[k] - a[k]; e2[k] = c[k] - a[k]; }
    }
    __device__ __forceinline__ float closest(const float* x, float* out) const { return closest_tri(x, a, e1, e2, out); }
    // watertight test in the sheared frame: the edge function of edge (P, Q)
    // is Q.x P.y - Q.y P.x from uncontracted products, so the two triangles
    // sharing an edge get exactly opposite values on it
    __device__ __forceinline__ float ray(const RaySetup<3>& r) const
    {
#pragma clang fp contract(off)
        float Ax, Ay, Az, Bx, By, Bz, Cx, Cy, Cz;
        r.shear(a, Ax, Ay, Az);
        r.shear(b, Bx, By, Bz);
        r.shear(c, Cx, Cy, Cz);
        const float U = Cx * By - Cy * Bx;
        const float V = Ax * Cy - Ay * Cx;
        const float W = Bx * Ay - By * Ax;
        if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return INFINITY;
        const float det = U + V + W;
        if (det == 0.f) return INFINITY;
        const float T = fmaf(U, Az, fmaf(V, Bz, W * Cz));
        return T / det;
    }
    // uniform point on the triangle from two uniforms
    __device__ __forceinline__ void point(float s1, float s2, float* z) const
    {
        const float sq = sqrtf(s1);
        const float u = sq * (1.f - s2), v = sq * s2;
#pragma unroll
        for (int i = 0; i < 3; ++i) z[i] = a[i] + u * e1[i] + v * e2[i];
    }
};

// ----------------------------------------------------------------- traversals
//
// Every query is resumable: its state is a small struct, begin() sets it up
// and step() visits one node (testing the primitives of leaf children
// inline), returning true once the query has finished.  A lane can therefore
// interleave queries of different walks; the run-to-completion functions
// further down loop over step(), so every caller runs the same code.

// Binary-tree traversal state: current node (-1 when finished), stack depth,
// best key so far and the primitive that attained it.
struct Trav {
    int node, sp;
    float best;
    int prim;
};

// After the children of a node were tested: descend into the live inner
// child with the smallest key and defer the others (farthest pushed first, so
// they come back nearest first), or resume from the deepest deferred entry
// whose key is still below `best`.  key[k] = +inf marks a child that is not
// followed.  Returns false when nothing is left.
__device__ __forceinline__ void sort_ce(float& ka, int& ra, float& kb, int& rb)
{
    const bool sw = kb < ka;
    const float tk = sw ? kb : ka;
    const int tr = sw ? rb : ra;
    kb = sw ? ka : kb;
    rb = sw ? ra : rb;
    ka = tk;
    ra = tr;
}

__device__ __forceinline__ bool trav_next4(float k0, float k1, float k2, float k3, const int4& ref, float best,
                                           Trav& q, const LdsStack& st)
{
    int r0 = ref.x, r1 = ref.y, r2 = ref.z, r3 = ref.w;
    sort_ce(k0, r0, k1, r1);
    sort_ce(k2, r2, k3, r3);
    sort_ce(k0, r0, k2, r2);
    sort_ce(k1, r1, k3, r3);
    sort_ce(k1, r1, k2, r2);
    if (k0 < INFINITY) {
        if (k3 < INFINITY) st.put(q.sp++, r3, k3);
        if (k2 < INFINITY) st.put(q.sp++, r2, k2);
        if (k1 < INFINITY) st.put(q.sp++, r1, k1);
        q.node = r0;
        return true;
    }
    while (q.sp > 0) {
        const uint2 e = st.get(--q.sp);
        if (__uint_as_float(e.y) < best) { q.node = (int)e.x; return true; }
    }
    q.node = -1;
    return false;
}

__device__ __forceinline__ void trav_begin(const DevBvh& b, float best, Trav& q)
{
    q.node = b.n_nodes > 0 ? 0 : -1;
    q.sp = 0;
    q.best = best;
    q.prim = -1;
}

// leaf children of a node whose key passes, as a bit mask
template <class F>
__device__ __forceinline__ uint32_t leaf_mask(const int4& ref, F pass)
{
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = comp(ref, k);
        if (r < 0 && r != kEmptyRef && pass(k)) m |= 1u << k;
    }
    return m;
}

// Takes the leaf child with the smallest key out of the mask lm.  Leaves are
// tested nearest first, so the first one usually sets the bound that lets the
// others go untested.
__device__ __forceinline__ int pop_nearest(uint32_t& lm, const float* key)
{
    int kb = 0;
    float kv = INFINITY;
    bool any = false;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (((lm >> k) & 1u) && (!any || key[k] < kv)) { kb = k; kv = key[k]; any = true; }
    lm &= ~(1u << kb);
    return kb;
}

// ---- closest Dirichlet point: q.best = squared distance, q.prim = primitive
template <int D, class S>
__device__ __forceinline__ bool closest_dirichlet_step(const DevBvh& b, const float* x, Trav& q, const LdsStack& st,
                                                       S* s)
{
    if (q.node < 0) return true;
    Node4<D> n;
    load_node4<D>(node_ptr<D>(b.nodes, q.node, Layout4<D>::kDirStride), n);
    stat_node(s);
    float key[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) key[k] = box_dist2<D>(n.box(k), x);   // empty children: +inf
    uint32_t lm = leaf_mask(n.ref, [&](int k) { return key[k] < q.best; });
    while (lm) {
        const int k = pop_nearest(lm, key);
        if (!(key[k] < q.best)) break;
        const int r = comp(n.ref, k);
        const int f = leaf_first(r), c = leaf_count(r);
        // a leaf's primitives are fetched four at a time and then tested in
        // order: one memory round trip per group instead of one per primitive
        for (int j0 = f; j0 < f + c; j0 += kPrimGroup) {
            Prim<D> pr[kPrimGroup];
#pragma unroll
            for (int u = 0; u < kPrimGroup; ++u)
                if (j0 + u < f + c) pr[u].load(b.prims, j0 + u);
#pragma unroll
            for (int u = 0; u < kPrimGroup; ++u) {
                if (j0 + u >= f + c) break;
                stat_prim(s);
                float cp[D];
                const float dd = pr[u].closest(x, cp);
                if (dd < q.best) { q.best = dd; q.prim = j0 + u; }
            }
        }
    }
    float kk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) kk[k] = comp(n.ref, k) >= 0 && key[k] < q.best ? key[k] : INFINITY;
    return !trav_next4(kk[0], kk[1], kk[2], kk[3], n.ref, q.best, q, st);
}

// ----------------------------------------------------------------- silhouettes

// true if the normal cone (axis, cos of the half-angle) of a child cannot
// contain a silhouette as seen from x: every primitive normal inside the cone
// makes an angle below pi/2 (all front) or above pi/2 (all back) with x - p
// for every p in the box.
template <int D>
__device__ __forceinline__ bool cone_culls(const Box<D>& b, const float4& cone, const float* x)
{
    // cone = (axis, cos theta).  With v = x - c for the box's bounding sphere
    // (centre c, radius R), every point p of the sphere and every normal n of
    // the cone keep (x - p).n of one sign iff the angle beta between v and the
    // axis stays more than theta + phi away from pi/2, phi = asin(R / |v|).
    // Without trigonometry: require theta + phi < pi/2 (R < |v| cos theta) and
    //   |v.axis| > |v| sin(theta + phi) = sin(theta) sqrt(|v|^2 - R^2) + cos(theta) R,
    // plus a margin of 1e-3 |v| (about 1e-3 rad of beta) for rounding.
    const float ct = cone.w;
    if (!(ct > 0.f)) return false;
    if constexpr (D == 2) {
        // In 2D the four corners are cheap and bound the box exactly: x - p
        // over the box is the convex hull of x - corner, and the directions
        // making an angle below pi/2 - theta with the axis (or above
        // pi/2 + theta) form a convex cone, so testing the corners decides
        // the whole box.  |d.axis| > (sin theta + 1e-3) |d| in squares.
        const float sm = sqrtf(fmaxf(1.f - ct * ct, 0.f)) + 1e-3f;
        const float sm2 = sm * sm;
        bool front = true, back = true;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float d0 = x[0] - ((c & 1) ? b.hi[0] : b.lo[0]);
            const float d1 = x[1] - ((c & 2) ? b.hi[1] : b.lo[1]);
            const float da = fmaf(d1, cone.y, d0 * cone.x);
            const bool out = da * da > sm2 * fmaf(d1, d1, d0 * d0);
            front = front && out && da > 0.f;
            back = back && out && da < 0.f;
        }
        return front || back;
    }
    float v[D], R2 = 0.f, dist2 = 0.f, va = 0.f;
    const float ax[3] = {cone.x, cone.y, cone.z};
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float h = 0.5f * (b.hi[i] - b.lo[i]);
        R2 = fmaf(h, h, R2);
        v[i] = x[i] - 0.5f * (b.lo[i] + b.hi[i]);
        dist2 = fmaf(v[i], v[i], dist2);
        va = fmaf(v[i], ax[i], va);
    }
    if (!(R2 < dist2 * ct * ct)) return false;
    const float st = sqrtf(fmaxf(1.f - ct * ct, 0.f));
    const float bound = fmaf(st, sqrtf(dist2 - R2), ct * sqrtf(R2)) + 1e-3f * sqrtf(dist2);
    return fabsf(va) > bound;
}

// Silhouette candidate k seen from x.  A Neumann primitive faces x from the
// front if x lies on its domain side; the primitive the walker stands on
// (internal id `onp`) is front by definition, every other facing decision is
// the exact sign.  Returns the squared distance if the candidate is a
// silhouette (adjacent primitives facing differently, or a boundary feature
// with a single adjacent Neumann primitive), +inf otherwise.
// the raw record of silhouette candidate k (2 float4 in 2D, 4 in 3D)
template <int D>
struct SilRec {
    float4 s[D == 2 ? 2 : 4];
    __device__ __forceinline__ void load(const float4* p, int k)
    {
#pragma unroll
        for (int i = 0; i < (D == 2 ? 2 : 4); ++i) s[i] = p[(D == 2 ? 2 : 4) * k + i];
    }
};

template <int D>
__device__ __forceinline__ float sil_rec_dist2(const SilRec<D>& r, const float* x, int onp)
{
    float a[D], n1[D], n2[D], e[D];
    int q1, q2;
    if (D == 2) {
        const float4 s0 = r.s[0], s1 = r.s[1];
        a[0] = s0.x; a[1] = s0.y; n1[0] = s0.z; n1[1] = s0.w;
        n2[0] = s1.x; n2[1] = s1.y;
        q1 = __float_as_int(s1.z); q2 = __float_as_int(s1.w);
    } else {
        const float4 s0 = r.s[0], s1 = r.s[1], s2 = r.s[D == 2 ? 0 : 2], s3 = r.s[D == 2 ? 1 : 3];
        a[0] = s0.x; a[1] = s0.y; a[2 % D] = s0.z;
        e[0] = s0.w - s0.x; e[1] = s1.x - s0.y; e[2 % D] = s1.y - s0.z;
        n1[0] = s1.z; n1[1] = s1.w; n1[2 % D] = s2.x;
        n2[0] = s2.y; n2[1] = s2.z; n2[2 % D] = s2.w;
        q1 = __float_as_int(s3.x); q2 = __float_as_int(s3.y);
    }
    float w[D];
#pragma unroll
    for (int i = 0; i < D; ++i) w[i] = x[i] - a[i];
    if (q2 >= 0) {
        const bool f1 = q1 == onp || dot<D>(w, n1) >= 0.f;
        const bool f2 = q2 == onp || dot<D>(w, n2) >= 0.f;
        if (f1 == f2) return INFINITY;
    }
    if (D == 2) return dot<D>(w, w);
    float c[D];
    return closest_seg<D>(x, a, e, c);
}

// ---- closest silhouette: q.best = squared distance (starts at the bound).
// `piece` is the convex piece of the Neumann primitive the walker stands on
// (-1 off the boundary or outside any piece): no candidate interior to that
// piece is a silhouette from x, so children holding only such candidates are
// skipped.
template <int D, class S>
__device__ __forceinline__ bool closest_silhouette_step(const DevBvh& b, const float* x, int onp, int piece,
                                                        Trav& q, const LdsStack& st, S* s)
{
    if (q.node < 0) return true;
    const float4* p = node_ptr<D>(b.nodes, q.node, Layout4<D>::kSilStride);
    Node4<D> n;
    load_node4<D>(p, n);
    float4 cn[D + 1];
#pragma unroll
    for (int a = 0; a <= D; ++a) cn[a] = p[Layout4<D>::kAux + a];
    const float4 pf = p[Layout4<D>::kPiece];
    const int4 pcs = make_int4(__float_as_int(pf.x), __float_as_int(pf.y), __float_as_int(pf.z), __float_as_int(pf.w));
    stat_node(s);
    float key[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const Box<D> bx = n.box(k);
        const float4 cone = make_float4(comp(cn[0], k), comp(cn[1], k), D == 3 ? comp(cn[D == 3 ? 2 : 0], k) : 0.f,
                                        comp(cn[D], k));
        const float d = box_dist2<D>(bx, x);
        const bool own = piece >= 0 && comp(pcs, k) == piece;
        key[k] = d < q.best && !own && !cone_culls<D>(bx, cone, x) ? d : INFINITY;
    }
    uint32_t lm = leaf_mask(n.ref, [&](int k) { return key[k] < q.best; });
    while (lm) {
        const int k = pop_nearest(lm, key);
        if (!(key[k] < q.best)) break;
        const int r = comp(n.ref, k);
        const int f = leaf_first(r), c = leaf_count(r);
        for (int j0 = f; j0 < f + c; j0 += kPrimGroup) {
            SilRec<D> rc[kPrimGroup];
#pragma unroll
            for (int u = 0; u < kPrimGroup; ++u)
                if (j0 + u < f + c) rc[u].load(b.prims, j0 + u);
#pragma unroll
            for (int u = 0; u < kPrimGroup; ++u) {
                if (j0 + u >= f + c) break;
                q.best = fminf(q.best, sil_rec_dist2<D>(rc[u], x, onp));
                stat_prim(s);
            }
        }
    }
    float kk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) kk[k] = comp(n.ref, k) >= 0 && key[k] < q.best ? key[k] : INFINITY;
    return !trav_next4(kk[0], kk[1], kk[2], kk[3], n.ref, q.best, q, st);
}

// ----------------------------------------------------------------- rays

// slab test: entry distance of the ray into the box within [tmin, tmax], or
// +inf.  The exit distance gets a relative slack of 1e-6 (a few roundings of
// the slab products), so a ray that meets a primitive is never rejected by a
// flat or grazed box around it.  tmin may be negative (crossings just behind
// the origin).
template <int D>
__device__ __forceinline__ float ray_box(const Box<D>& b, const float* x, const float* inv, float tmin, float tmax)
{
    float t0 = tmin, t1 = tmax;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float a = (b.lo[i] - x[i]) * inv[i];
        const float c = (b.hi[i] - x[i]) * inv[i];
        t0 = fmaxf(t0, fminf(a, c));
        t1 = fminf(t1, fmaxf(a, c));
    }
    return t0 <= t1 + 1e-6f * fabsf(t1) ? t0 : INFINITY;
}

// true if direction nu leaves the domain through Neumann primitive k
template <int D>
__device__ __forceinline__ bool exits(const DevBvh& b, int k, const float* nu)
{
    const float4 e = b.pextra[k];
    const float no[3] = {e.x, e.y, e.z};
    return dot<D>(no, nu) > 0.f;
}

// Ray state: traversal state plus the reciprocal direction of the slabs.
// q.best = nearest accepted t, q.prim = hit primitive.
template <int D>
struct RayTrav {
    Trav t;
    float inv[D];
};

template <int D>
__device__ __forceinline__ void ray_begin(const DevBvh& b, const float* nu, float tmax, RayTrav<D>& q)
{
    trav_begin(b, tmax, q.t);
#pragma unroll
    for (int i = 0; i < D; ++i) q.inv[i] = 1.f / nu[i];
}

// ---- first Neumann hit with t in (tau, tmax), skipping internal primitive
// `skip`.  Walk rays pass tau = 0: a walker standing on the boundary shoots
// from an origin offset along its normal instead, so no genuine crossing near
// the origin is ever ignored.  With back > 0 a crossing at t in (-back, tau]
// also counts if the ray leaves the domain through it (nu . n_out > 0): seen
// from inside, the first crossing is always an exit, so an exit at or just
// behind the origin means the origin lies on the boundary up to rounding, and
// the walker is put back onto it.
template <int D, class S>
__device__ __forceinline__ bool ray_neumann_step(const DevBvh& b, const float* x, const float* nu, float tau,
                                                 float back, int skip, RayTrav<D>& q, const LdsStack& st, S* s)
{
    if (q.t.node < 0) return true;
    const RaySetup<D> ry(x, nu);
    Node4<D> n;
    load_node4<D>(node_ptr<D>(b.nodes, q.t.node, Layout4<D>::kNeuStride), n);
    stat_node(s);
    float key[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        key[k] = comp(n.ref, k) != kEmptyRef ? ray_box<D>(n.box(k), x, q.inv, -back, q.t.best) : INFINITY;
    uint32_t lm = leaf_mask(n.ref, [&](int k) { return key[k] < INFINITY; });
    while (lm) {
        // nearest entry first; a leaf entered beyond the best hit holds no
        // nearer one (the slab slack keeps every crossing inside its box)
        const int k = pop_nearest(lm, key);
        if (!(key[k] <= q.t.best)) break;
        const int r = comp(n.ref, k);
        const int f = leaf_first(r), c = leaf_count(r);
        for (int j = f; j < f + c; ++j) {
            if (j == skip) continue;
            Prim<D> pr; pr.load(b.prims, j); stat_prim(s);
            const float t = pr.ray(ry);
            if (t < q.t.best && (t > tau || (t > -back && exits<D>(b, j, nu)))) { q.t.best = t; q.t.prim = j; }
        }
    }
    float kk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) kk[k] = comp(n.ref, k) >= 0 && key[k] < q.t.best ? key[k] : INFINITY;
    return !trav_next4(kk[0], kk[1], kk[2], kk[3], n.ref, q.t.best, q.t, st);
}

// ---- visibility: does a Neumann primitive other than `skip` and `skip2`
// cross the ray x + t nu (unit nu) at t in (t_lo, t_hi)?  Any-hit: finishes
// at the first blocker, with q.t.prim >= 0; q.t.best holds t_hi.  A ray
// toward a point on a primitive skips that primitive: a flat primitive meets
// the segment to one of its points only there, and at the grazing angles of
// rays along the boundary the FP32 crossing parameter of the target's own
// primitive can land well short of the end of the ray.
template <int D, class S>
__device__ __forceinline__ bool visible_neumann_step(const DevBvh& b, const float* x, const float* nu, float t_lo,
                                                     int skip, int skip2, RayTrav<D>& q, const LdsStack& st, S* s)
{
    if (q.t.node < 0) return true;
    const RaySetup<D> ry(x, nu);
    const float tmax = q.t.best;
    Node4<D> n;
    load_node4<D>(node_ptr<D>(b.nodes, q.t.node, Layout4<D>::kNeuStride), n);
    stat_node(s);
    float key[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        key[k] = comp(n.ref, k) != kEmptyRef ? ray_box<D>(n.box(k), x, q.inv, 0.f, tmax) : INFINITY;
    uint32_t lm = leaf_mask(n.ref, [&](int k) { return key[k] < INFINITY; });
    while (lm) {
        const int k = __builtin_ctz(lm);
        lm &= lm - 1;
        const int r = comp(n.ref, k);
        const int f = leaf_first(r), c = leaf_count(r);
        for (int j = f; j < f + c; ++j) {
            if (j == skip || j == skip2) continue;
            Prim<D> pr; pr.load(b.prims, j); stat_prim(s);
            const float t = pr.ray(ry);
            if (t > t_lo && t < tmax) { q.t.prim = j; q.t.node = -1; return true; }
        }
    }
    float kk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) kk[k] = comp(n.ref, k) >= 0 ? key[k] : INFINITY;
    return !trav_next4(kk[0], kk[1], kk[2], kk[3], n.ref, INFINITY, q.t, st);
}

// ----------------------------------------------------------------- Neumann sample

// Pick one Neumann primitive meeting the ball B(x, r): descend choosing each
// child with probability proportional to its subtree measure (children whose
// box misses the ball get weight 0), then a primitive of the leaf in
// proportion to its measure among the leaf primitives meeting the ball.
// State: node (-1 when finished), the running uniform u, the probability of
// the path so far, and the result (prim, prob).
struct SampleTrav {
    int node;
    float u, P;
    int prim;
    float prob;
};

__device__ __forceinline__ void sample_begin(const DevBvh& b, float u, SampleTrav& q)
{
    q.node = b.n_nodes > 0 ? 0 : -1;
    q.u = u;
    q.P = 1.f;
    q.prim = -1;
    q.prob = 0.f;
}

template <int D, class S>
__device__ __forceinline__ bool sample_neumann_step(const DevBvh& b, const float* x, float r, SampleTrav& q, S* s)
{
    if (q.node < 0) return true;
    const float r2 = r * r;
    const float4* p = node_ptr<D>(b.nodes, q.node, Layout4<D>::kNeuStride);
    Node4<D> n;
    load_node4<D>(p, n);
    const float4 meas = p[Layout4<D>::kAux];
    stat_node(s);
    // children whose box misses the ball get weight 0 (empty children have
    // an empty box and measure 0)
    float w[4], W = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w[k] = box_dist2<D>(n.box(k), x) < r2 ? comp(meas, k) : 0.f;
        W += w[k];
    }
    if (!(W > 0.f)) { q.node = -1; return true; }
    // child k with probability w_k / W: the first whose running sum exceeds
    // u W (the last positive one if rounding leaves none)
    const float t = q.u * W;
    float lo = 0.f, acc = 0.f, wk = 0.f;
    int ck = 0;
    bool found = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float a0 = acc;
        acc += w[k];
        if (w[k] > 0.f && !found) { ck = k; lo = a0; wk = w[k]; found = t < acc; }
    }
    q.P *= wk / W;
    const float u = fminf(fmaxf((t - lo) / wk, 0.f), 0.99999994f);
    q.u = u;
    const int rf = comp(n.ref, ck);
    if (rf >= 0) { q.node = rf; return false; }
    const int c = leaf_first(rf), nn = leaf_count(rf);
    // leaf: measure-weighted choice among primitives meeting the ball
    q.node = -1;
    float tot = 0.f;
    for (int k = c; k < c + nn; ++k) {
        Prim<D> pr; pr.load(b.prims, k); stat_prim(s);
        float z[D];
        if (pr.closest(x, z) < r2) tot += b.pextra[k].w;
    }
    if (!(tot > 0.f)) return true;
    const float target = u * tot;
    float acc2 = 0.f;
    int sel = -1;
    float wsel = 0.f;
    for (int k = c; k < c + nn; ++k) {
        Prim<D> pr; pr.load(b.prims, k); stat_prim(s);
        float z[D];
        if (!(pr.closest(x, z) < r2)) continue;
        const float wj = b.pextra[k].w;
        sel = k; wsel = wj;
        acc2 += wj;
        if (target < acc2) break;
    }
    q.prim = sel;
    q.prob = q.P * (wsel / tot);
    return true;
}

// ----------------------------------------------------------------- run to completion

// Squared distance to the closest Dirichlet point (best2 on entry bounds the
// search), the point itself and its internal primitive (-1 if none found).
template <int D, class S = NoStat>
__device__ float closest_dirichlet(const DevBvh& b, const float* x, float best2, float* xbar, int* prim_out,
                                   const LdsStack& st, S* s = nullptr)
{
    Trav q;
    trav_begin(b, best2, q);
    while (!closest_dirichlet_step<D>(b, x, q, st, s)) {}
    *prim_out = q.prim;
    if (q.prim >= 0) {
        Prim<D> pr;
        pr.load(b.prims, q.prim);
        pr.closest(x, xbar);
    }
    return q.best;
}

template <int D, class S = NoStat>
__device__ float closest_silhouette(const DevBvh& b, const float* x, float best2, int onp, const LdsStack& st,
                                    S* s = nullptr)
{
    Trav q;
    trav_begin(b, best2, q);
    const int piece = onp >= 0 && b.piece ? b.piece[onp] : -1;
    while (!closest_silhouette_step<D>(b, x, onp, piece, q, st, s)) {}
    return q.best;
}

template <int D, class S = NoStat>
__device__ float ray_neumann(const DevBvh& b, const float* x, const float* nu, float tmax, float tau, int skip,
                             int* hit, const LdsStack& st, S* s = nullptr, float back = 0.f)
{
    RayTrav<D> q;
    ray_begin<D>(b, nu, tmax, q);
    while (!ray_neumann_step<D>(b, x, nu, tau, back, skip, q, st, s)) {}
    *hit = q.t.prim;
    return q.t.prim >= 0 ? q.t.best : INFINITY;
}

template <int D, class S = NoStat>
__device__ bool visible_neumann(const DevBvh& b, const float* x, const float* nu, float t_lo, float t_hi, int skip,
                                int skip2, const LdsStack& st, S* s = nullptr)
{
    RayTrav<D> q;
    ray_begin<D>(b, nu, t_hi, q);
    while (!visible_neumann_step<D>(b, x, nu, t_lo, skip, skip2, q, st, s)) {}
    return q.t.prim < 0;
}

template <int D, class S = NoStat>
__device__ int sample_neumann(const DevBvh& b, const float* x, float r, float u, float* prob, S* s = nullptr)
{
    SampleTrav q;
    sample_begin(b, u, q);
    while (!sample_neumann_step<D>(b, x, r, q, s)) {}
    *prob = q.prob;
    return q.prim;
}

}  // namespace wost
