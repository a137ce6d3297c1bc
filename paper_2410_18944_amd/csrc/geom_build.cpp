// Host-side construction of the walk-on-stars boundary hierarchies
// (wost_build_bvh) and their upload into caller-owned device memory.
//
// Three binary hierarchies are built with object-median splits along the
// longest centroid extent (depth <= ceil(log2(n / leaf)) + 1) and stored
// four-wide: each node holds the children of a binary node, every inner
// child replaced by its own two children (the layout is in wost_internal.h):
//   * Dirichlet primitives  -> closest point + epsilon-shell test (Sec. 3.2)
//   * Neumann primitives    -> first hit inside the star, visibility, and the
//                              area-weighted Neumann sample (node measures)
//   * Neumann silhouette candidates (2D vertices, 3D edges) with the inward
//     normals of their adjacent Neumann primitives, per-child normal cones
//     and, in 2D, the convex piece of the boundary each candidate is interior
//     to -> distance to the closest silhouette, which bounds the star radius
//     (Sec. 3.2).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "wost_internal.h"

namespace wost {

static thread_local std::string g_err;

void set_error(const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

namespace {

struct Box {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void add(const double* p, int d)
    {
        for (int i = 0; i < d; ++i) { lo[i] = std::min(lo[i], p[i]); hi[i] = std::max(hi[i], p[i]); }
    }
    void add(const Box& b, int d)
    {
        for (int i = 0; i < d; ++i) { lo[i] = std::min(lo[i], b.lo[i]); hi[i] = std::max(hi[i], b.hi[i]); }
    }
};

// One item of a hierarchy: its box, centroid, and payload index.
struct Item {
    Box box;
    double c[3];
    int32_t id;
};

struct BuiltNode {
    Box box[2];
    int32_t c[2] = {-1, -1};
    int32_t n[2] = {0, 0};
};

struct Builder {
    int d;
    int leaf;
    bool brute;
    std::vector<Item>* items;
    std::vector<BuiltNode> nodes;
    std::vector<int32_t> order;       // leaf order of item ids
    int max_depth = 0;

    Box range_box(int b, int e) const
    {
        Box bx;
        for (int i = b; i < e; ++i) bx.add((*items)[i].box, d);
        return bx;
    }

    // returns (c, n) describing the subtree over items[b, e)
    void build(int b, int e, int depth, int32_t& out_c, int32_t& out_n)
    {
        max_depth = std::max(max_depth, depth);
        if (e - b <= leaf) {
            // a leaf lists its items by id, whatever order the splits left
            std::sort(items->begin() + b, items->begin() + e,
                      [](const Item& p, const Item& q) { return p.id < q.id; });
            out_c = (int32_t)order.size();
            out_n = e - b;
            for (int i = b; i < e; ++i) order.push_back((*items)[i].id);
            return;
        }
        Box cb;
        for (int i = b; i < e; ++i) cb.add((*items)[i].c, d);
        int ax = 0;
        for (int i = 1; i < d; ++i)
            if (cb.hi[i] - cb.lo[i] > cb.hi[ax] - cb.lo[ax]) ax = i;
        int m = (b + e) / 2;
        std::nth_element(items->begin() + b, items->begin() + m, items->begin() + e,
                         [ax](const Item& p, const Item& q) {
                             if (p.c[ax] != q.c[ax]) return p.c[ax] < q.c[ax];
                             return p.id < q.id;
                         });
        int32_t idx = (int32_t)nodes.size();
        nodes.emplace_back();
        int32_t c0, n0, c1, n1;
        build(b, m, depth + 1, c0, n0);
        build(m, e, depth + 1, c1, n1);
        BuiltNode& nd = nodes[idx];
        nd.box[0] = range_box(b, m);
        nd.box[1] = range_box(m, e);
        nd.c[0] = c0; nd.n[0] = n0; nd.c[1] = c1; nd.n[1] = n1;
        out_c = idx;
        out_n = 0;
    }

    // Build; guarantees a root node (index 0) exists when there are items.
    void run()
    {
        int n = (int)items->size();
        if (n == 0) return;
        int32_t c, k;
        if (n <= leaf) {
            nodes.emplace_back();
            build(0, n, 1, c, k);
            nodes[0].box[0] = range_box(0, n);
            nodes[0].c[0] = c; nodes[0].n[0] = k;
            return;
        }
        build(0, n, 0, c, k);
        // build() placed the root at index 0
    }
};

struct Sil {
    double a[3], b[3];      // 2D: vertex in a (b = a)
    double n1[3], n2[3];    // inward normals of adjacent Neumann prims; n2 = 0 if boundary
    bool boundary;
    int64_t q1, q2;         // adjacent Neumann primitives (caller ids); q2 = -1 if boundary
    int64_t v;              // 2D: vertex id
    int32_t piece;          // convex piece the vertex is interior to, or -1
};

inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

}  // namespace

}  // namespace wost

using namespace wost;

namespace {

template <class T>
int64_t push_bytes(std::vector<uint8_t>& img, const T* data, size_t count)
{
    size_t off = (img.size() + 255) & ~size_t(255);
    img.resize(off + sizeof(T) * count);
    if (count) memcpy(img.data() + off, data, sizeof(T) * count);
    return (int64_t)off;
}

}  // namespace

wost::DevGeom wost_geom::devgeom() const
{
    DevGeom g{};
    const uint8_t* base = (const uint8_t*)dev;
    DevBvh* b[3] = {&g.dir, &g.neu, &g.sil};
    for (int i = 0; i < 3; ++i) {
        b[i]->nodes = (const float4*)(base + sec[i].nodes);
        b[i]->prims = (const float4*)(base + sec[i].prims);
        b[i]->pextra = sec[i].pextra >= 0 ? (const float4*)(base + sec[i].pextra) : nullptr;
        b[i]->orig = sec[i].orig >= 0 ? (const int32_t*)(base + sec[i].orig) : nullptr;
        b[i]->piece = sec[i].piece >= 0 ? (const int32_t*)(base + sec[i].piece) : nullptr;
        b[i]->n_nodes = sec[i].n_nodes;
        b[i]->n_prims = sec[i].n_prims;
    }
    if (dir_dev.nodes) {
        g.dir.nodes = (const float4*)dir_dev.nodes;
        g.dir.prims = (const float4*)dir_dev.prims;
        g.dir.pextra = nullptr;
        g.dir.orig = dir_dev.orig;
        g.dir.piece = nullptr;
        g.dir.n_nodes = dir_dev.n_nodes;
        g.dir.n_prims = dir_dev.n_prims;
    }
    g.neu_id = off_neu_id >= 0 ? (const int32_t*)(base + off_neu_id) : nullptr;
    g.n_caller = n_caller;
    g.dim = dim;
    g.diag = (float)diag;
    g.tau = (float)(1e-6 * diag);
    for (int i = 0; i < 3; ++i) { g.lo[i] = (float)lo[i]; g.hi[i] = (float)hi[i]; }
    return g;
}

extern "C" const char* wost_last_error(void) { return wost::g_err.c_str(); }

extern "C" int wost_geom_use_dirichlet_lbvh(wost_geom* g, const float* nodes, int32_t n_nodes,
                                           const float* prims_sorted, const int32_t* orig, int32_t n_prims,
                                           int32_t levels)
{
    if (!g) { set_error("wost_geom_use_dirichlet_lbvh: NULL geometry"); return WOST_EINVAL; }
    if (!nodes) {
        g->dir_dev = wost_geom::DirDev{};
        return WOST_OK;
    }
    if (!prims_sorted || !orig || n_nodes < 1 || levels < 1) {
        set_error("wost_geom_use_dirichlet_lbvh: need nodes, sorted primitives, orig, n_nodes >= 1, levels >= 1");
        return WOST_EINVAL;
    }
    if (n_prims != g->n_dir) {
        set_error("wost_geom_use_dirichlet_lbvh: %d primitives, the geometry has %lld Dirichlet primitives", n_prims,
                  (long long)g->n_dir);
        return WOST_EINVAL;
    }
    const int64_t stack = 3 * ((int64_t)levels - 1) + 1;
    if (stack > kMaxStack) {
        set_error("wost_geom_use_dirichlet_lbvh: %d levels need %lld stack entries (at most %d)", levels,
                  (long long)stack, kMaxStack);
        return WOST_EUNSUPPORTED;
    }
    g->dir_dev.nodes = nodes;
    g->dir_dev.prims = prims_sorted;
    g->dir_dev.orig = orig;
    g->dir_dev.n_nodes = n_nodes;
    g->dir_dev.n_prims = n_prims;
    g->dir_dev.stack = (int32_t)stack;
    return WOST_OK;
}

extern "C" int wost_build_bvh(int32_t dim, const float* verts, int64_t n_verts, const int32_t* prims,
                              int64_t n_prims, const uint8_t* bc, const wost_build_opts* opts,
                              wost_geom** out)
{
    if (!out) { set_error("wost_build_bvh: out is NULL"); return WOST_EINVAL; }
    *out = nullptr;
    if (dim != 2 && dim != 3) { set_error("wost_build_bvh: dim must be 2 or 3 (got %d)", dim); return WOST_EINVAL; }
    if (!verts || !prims || !bc || n_verts <= 0 || n_prims <= 0) {
        set_error("wost_build_bvh: empty or NULL geometry");
        return WOST_EINVAL;
    }
    if (n_prims >= (1ll << 30) || n_verts >= (1ll << 31)) {
        set_error("wost_build_bvh: too many primitives");
        return WOST_EUNSUPPORTED;
    }
    int leaf = 4;
    bool brute = false;
    if (opts) {
        if (opts->leaf_size < 1 || opts->leaf_size > 64) {
            set_error("wost_build_bvh: leaf_size must be in [1, 64]");
            return WOST_EINVAL;
        }
        leaf = opts->leaf_size;
        brute = opts->brute_force != 0;
    }
    const int d = dim;
    // ---- per-primitive data in double
    std::vector<double> P((size_t)n_prims * d * d);
    std::vector<std::array<double, 3>> nout(n_prims);
    std::vector<double> meas(n_prims);
    Box all;
    for (int64_t v = 0; v < n_verts; ++v) {
        double p[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) {
            p[i] = verts[v * d + i];
            if (!std::isfinite(p[i])) { set_error("wost_build_bvh: non-finite vertex %lld", (long long)v); return WOST_EINVAL; }
        }
        all.add(p, d);
    }
    for (int i = 0; i < 3; ++i) { all.lo[i] += 0.0; all.hi[i] += 0.0; }   // no negative zeros
    for (int64_t q = 0; q < n_prims; ++q) {
        if (bc[q] > 1) { set_error("wost_build_bvh: bc[%lld] must be 0 or 1", (long long)q); return WOST_EINVAL; }
        for (int k = 0; k < d; ++k) {
            int32_t vid = prims[q * d + k];
            if (vid < 0 || vid >= n_verts) {
                set_error("wost_build_bvh: prim %lld references vertex %d out of range", (long long)q, vid);
                return WOST_EINVAL;
            }
            for (int i = 0; i < d; ++i) P[(q * d + k) * d + i] = verts[(int64_t)vid * d + i];
        }
        const double* a = &P[q * d * d];
        if (d == 2) {
            double ex = a[2] - a[0], ey = a[3] - a[1];
            double len = std::sqrt(ex * ex + ey * ey);
            if (!(len > 0)) { set_error("wost_build_bvh: degenerate segment %lld", (long long)q); return WOST_EINVAL; }
            nout[q] = {ey / len, -ex / len, 0.0};
            meas[q] = len;
        } else {
            double e1[3], e2[3];
            for (int i = 0; i < 3; ++i) { e1[i] = a[3 + i] - a[i]; e2[i] = a[6 + i] - a[i]; }
            double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
            double len = std::sqrt(dot3(c, c));
            if (!(len > 0)) { set_error("wost_build_bvh: degenerate triangle %lld", (long long)q); return WOST_EINVAL; }
            nout[q] = {c[0] / len, c[1] / len, c[2] / len};
            meas[q] = 0.5 * len;
        }
    }
    auto prim_box = [&](int64_t q) {
        Box b;
        for (int k = 0; k < d; ++k) b.add(&P[(q * d + k) * d], d);
        return b;
    };
    // ---- silhouette candidates
    std::vector<Sil> sils;
    {
        std::map<std::pair<int64_t, int64_t>, std::vector<int64_t>> adj;
        for (int64_t q = 0; q < n_prims; ++q) {
            if (!bc[q]) continue;
            if (d == 2) {
                for (int k = 0; k < 2; ++k) adj[{prims[q * 2 + k], -1}].push_back(q);
            } else {
                for (int k = 0; k < 3; ++k) {
                    int64_t a = prims[q * 3 + k], b = prims[q * 3 + (k + 1) % 3];
                    adj[{std::min(a, b), std::max(a, b)}].push_back(q);
                }
            }
        }
        sils.reserve(adj.size());
        for (auto& kv : adj) {
            Sil s{};
            int64_t va = kv.first.first, vb = kv.first.second < 0 ? va : kv.first.second;
            for (int i = 0; i < d; ++i) { s.a[i] = verts[va * d + i]; s.b[i] = verts[vb * d + i]; }
            const auto& L = kv.second;
            for (int i = 0; i < 3; ++i) s.n1[i] = -nout[L[0]][i];
            s.boundary = L.size() < 2;
            s.q1 = L[0];
            s.q2 = s.boundary ? -1 : L[1];
            for (int i = 0; i < 3; ++i) s.n2[i] = s.boundary ? 0.0 : -nout[L[1]][i];
            s.v = va;
            s.piece = -1;
            sils.push_back(s);
        }
    }
    // ---- convex pieces (2D).  A vertex shared by exactly two Neumann
    // segments links them when it is strictly convex, one segment ends where
    // the other starts, and both outward normals lie in the same closed
    // quadrant.  A piece is a maximal chain of links: its normals turn one
    // way by at most pi/2, so it is the graph of a convex function over some
    // direction and lies on the domain side of every one of its segments'
    // lines.  Seen from a point on one of its segments every segment of the
    // piece faces front, and no vertex interior to it is a silhouette.  A
    // piece is named by the caller index of its last segment, found by
    // pointer jumping along the links for a fixed number of rounds (a closed
    // chain, impossible for these turns, would only split into more names).
    std::vector<int32_t> seg_piece(n_prims, -1);
    std::vector<char> link(d == 2 ? n_verts : 0, 0);
    if (d == 2) {
        std::vector<std::vector<int64_t>> inc(n_verts);
        for (int64_t q = 0; q < n_prims; ++q)
            if (bc[q])
                for (int k = 0; k < 2; ++k) inc[prims[q * 2 + k]].push_back(q);
        auto quadrant = [&](int64_t q) {
            return nout[q][0] >= 0 ? (nout[q][1] >= 0 ? 0 : 3) : (nout[q][1] >= 0 ? 1 : 2);
        };
        std::vector<int64_t> jump(n_prims, -1), jump2(n_prims, -1);
        int64_t n_neu_segs = 0;
        for (int64_t q = 0; q < n_prims; ++q)
            if (bc[q]) { jump[q] = q; ++n_neu_segs; }
        for (int64_t v = 0; v < n_verts; ++v) {
            if (inc[v].size() != 2) continue;
            const int64_t s1 = inc[v][0], s2 = inc[v][1];
            const bool end1 = prims[s1 * 2 + 1] == v, end2 = prims[s2 * 2 + 1] == v;
            if (end1 == end2) continue;
            const int64_t p1 = end1 ? prims[s1 * 2] : prims[s1 * 2 + 1];
            const int64_t p2 = end2 ? prims[s2 * 2] : prims[s2 * 2 + 1];
            double e1[2], e2[2];
            for (int i = 0; i < 2; ++i) {
                e1[i] = (double)verts[p1 * 2 + i] - (double)verts[v * 2 + i];
                e2[i] = (double)verts[p2 * 2 + i] - (double)verts[v * 2 + i];
            }
            const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1]);
            const double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1]);
            // sine of the turn, measured against each outward normal
            const double c1 = -(e2[0] * nout[s1][0] + e2[1] * nout[s1][1]) / l2;
            const double c2 = -(e1[0] * nout[s2][0] + e1[1] * nout[s2][1]) / l1;
            if (!(c1 > 1e-6 && c2 > 1e-6) || quadrant(s1) != quadrant(s2)) continue;
            link[v] = 1;
            if (end1) jump[s1] = s2;
            else jump[s2] = s1;
        }
        int rounds = 1;
        while ((int64_t(1) << rounds) < n_neu_segs + 1) ++rounds;
        for (int r = 0; r < rounds; ++r) {
            for (int64_t q = 0; q < n_prims; ++q) jump2[q] = jump[q] >= 0 ? jump[jump[q]] : -1;
            jump.swap(jump2);
        }
        for (int64_t q = 0; q < n_prims; ++q) seg_piece[q] = bc[q] ? (int32_t)jump[q] : -1;
        for (auto& sl : sils)
            if (link[sl.v]) sl.piece = seg_piece[sl.q1];
    }
    // ---- hierarchies
    wost_geom* g = new wost_geom();
    g->dim = d;
    for (int i = 0; i < 3; ++i) { g->lo[i] = i < d ? all.lo[i] : 0; g->hi[i] = i < d ? all.hi[i] : 0; }
    double diag2 = 0;
    for (int i = 0; i < d; ++i) diag2 += (all.hi[i] - all.lo[i]) * (all.hi[i] - all.lo[i]);
    g->diag = std::sqrt(diag2);
    std::vector<uint8_t> img;
    std::vector<int32_t> orig_all;
    std::vector<int32_t> neu_internal(n_prims, -1);   // caller id -> internal Neumann id
    auto int_bits = [](int32_t v) { float f; memcpy(&f, &v, 4); return f; };

    for (int which = 0; which < 3; ++which) {
        std::vector<Item> items;
        if (which < 2) {
            for (int64_t q = 0; q < n_prims; ++q) {
                if ((int)bc[q] != which) continue;
                Item it;
                it.box = prim_box(q);
                for (int i = 0; i < 3; ++i) it.c[i] = 0.5 * (it.box.lo[i] + it.box.hi[i]);
                for (int i = d; i < 3; ++i) it.c[i] = 0;
                it.id = (int32_t)q;
                items.push_back(it);
            }
        } else {
            for (size_t k = 0; k < sils.size(); ++k) {
                Item it;
                it.box.add(sils[k].a, d);
                it.box.add(sils[k].b, d);
                for (int i = 0; i < 3; ++i) it.c[i] = i < d ? 0.5 * (it.box.lo[i] + it.box.hi[i]) : 0;
                it.id = (int32_t)k;
                items.push_back(it);
            }
        }
        // brute force: leaves of the maximum size whose boxes all cover the
        // whole hierarchy and cones that never cull, so every query tests
        // every primitive
        Builder B{d, brute ? kLeafMax : leaf, brute, &items, {}, {}, 0};
        B.run();
        g->max_depth = std::max(g->max_depth, B.max_depth);
        const int nn = (int)B.nodes.size();
        const int np = (int)B.order.size();
        // structural validation: every child reference in range, every item in
        // exactly one leaf (the kernels index without further checks)
        {
            std::vector<int> seen(np, 0);
            bool ok = np == (int)items.size() && (nn > 0 || np == 0);
            for (int ni = 0; ni < nn && ok; ++ni) {
                for (int ch = 0; ch < 2 && ok; ++ch) {
                    const int c = B.nodes[ni].c[ch], n = B.nodes[ni].n[ch];
                    if (n > 0) {
                        ok = c >= 0 && c + n <= np;
                        for (int k = c; ok && k < c + n; ++k) seen[k]++;
                    } else if (c >= 0) {
                        ok = c > ni && c < nn;
                    } else {
                        ok = ch == 1 && ni == 0;   // only the root's second child may be empty
                    }
                }
            }
            for (int k = 0; k < np && ok; ++k) ok = seen[k] == 1;
            if (!ok) {
                set_error("wost_build_bvh: internal error: hierarchy %d failed validation", which);
                delete g;
                return WOST_EINVAL;
            }
        }
        // aggregates per node child, bottom-up (children are created after
        // their parents): the Neumann measure of the subtree; for
        // silhouettes the sum of the candidates' normals (a leaf adds its
        // candidates' normals in leaf order, an inner child copies its node's
        // sum, and a node adds its two children's sums), how many normals,
        // whether a boundary feature lies below, and the convex piece all
        // candidates share
        std::vector<double> sub_meas(nn * 2, 0.0), node_meas(nn, 0.0);
        std::vector<std::array<double, 3>> sub_sum(which == 2 ? nn * 2 : 0), node_sum(which == 2 ? nn : 0);
        std::vector<int64_t> sub_cnt(which == 2 ? nn * 2 : 0, 0), node_cnt(which == 2 ? nn : 0, 0);
        std::vector<char> sub_bnd(which == 2 ? nn * 2 : 0, 0), node_bnd(which == 2 ? nn : 0, 0);
        // leaf-order range [first, first + count) of every child
        std::vector<int32_t> sub_first(nn * 2, 0), sub_count(nn * 2, 0), node_first(nn, 0), node_count(nn, 0);
        std::vector<int32_t> sub_piece(nn * 2, -1), node_piece(nn, -1);
        auto join_piece = [](int32_t a, int32_t b) { return a == -2 ? b : (b == -2 ? a : (a == b ? a : -1)); };
        for (int ni = nn - 1; ni >= 0; --ni) {
            const BuiltNode& nd = B.nodes[ni];
            int32_t np_acc = -2;
            double nsum[3] = {0.0, 0.0, 0.0};
            for (int ch = 0; ch < 2; ++ch) {
                const int k2 = ni * 2 + ch;
                double m = 0;
                double ssum[3] = {0.0, 0.0, 0.0};
                int64_t cnt = 0;
                bool bnd = false;
                int32_t pc = -2;
                if (nd.n[ch] > 0) {
                    sub_first[k2] = nd.c[ch];
                    sub_count[k2] = nd.n[ch];
                    for (int k = nd.c[ch]; k < nd.c[ch] + nd.n[ch]; ++k) {
                        const int32_t id = B.order[k];
                        if (which == 1) m += meas[id];
                        if (which == 2) {
                            const Sil& sl = sils[id];
                            for (int i = 0; i < 3; ++i) ssum[i] += sl.n1[i];
                            ++cnt;
                            if (!sl.boundary) {
                                for (int i = 0; i < 3; ++i) ssum[i] += sl.n2[i];
                                ++cnt;
                            }
                            bnd = bnd || sl.boundary;
                            pc = join_piece(pc, sl.piece);
                        }
                    }
                } else if (nd.c[ch] >= 0) {
                    const int c = nd.c[ch];
                    sub_first[k2] = node_first[c];
                    sub_count[k2] = node_count[c];
                    m = node_meas[c];
                    if (which == 2) {
                        for (int i = 0; i < 3; ++i) ssum[i] = node_sum[c][i];
                        cnt = node_cnt[c];
                        bnd = node_bnd[c];
                        pc = node_piece[c];
                    }
                }
                sub_meas[k2] = m;
                node_meas[ni] += m;
                node_count[ni] += sub_count[k2];
                if (which == 2) {
                    for (int i = 0; i < 3; ++i) { sub_sum[k2][i] = ssum[i]; nsum[i] += ssum[i]; }
                    sub_cnt[k2] = cnt;
                    sub_bnd[k2] = bnd;
                    sub_piece[k2] = pc == -2 ? -1 : pc;
                    node_cnt[ni] += cnt;
                    node_bnd[ni] = node_bnd[ni] || bnd;
                    np_acc = join_piece(np_acc, pc);
                }
            }
            node_first[ni] = sub_first[ni * 2];
            if (which == 2) {
                for (int i = 0; i < 3; ++i) node_sum[ni][i] = nsum[i];
                node_piece[ni] = np_acc == -2 ? -1 : np_acc;
            }
        }
        // normal cone of every child: axis = normalised normal sum, and the
        // cosine of its half-angle = the smallest cosine between the axis and
        // any normal below (from 1); undefined sums give the axis (1, 0, 0)
        // and a cone that never culls
        std::vector<std::array<double, 4>> sub_cone(which == 2 ? nn * 2 : 0, {1.0, 0.0, 0.0, -1.0});
        if (which == 2) {
            for (int k2 = 0; k2 < nn * 2; ++k2) {
                const auto& sm = sub_sum[k2];
                const double len = std::sqrt(sm[0] * sm[0] + sm[1] * sm[1] + sm[2] * sm[2]);
                if (sub_cnt[k2] == 0 || len < 1e-9 * (double)sub_cnt[k2]) continue;
                const double ax[3] = {sm[0] / len, sm[1] / len, sm[2] / len};
                double worst = 1.0;
                for (int k = sub_first[k2]; k < sub_first[k2] + sub_count[k2]; ++k) {
                    const Sil& sl = sils[B.order[k]];
                    worst = std::min(worst, ax[0] * sl.n1[0] + ax[1] * sl.n1[1] + ax[2] * sl.n1[2]);
                    if (!sl.boundary) worst = std::min(worst, ax[0] * sl.n2[0] + ax[1] * sl.n2[1] + ax[2] * sl.n2[2]);
                }
                sub_cone[k2] = {ax[0], ax[1], ax[2], worst};
            }
        }
        // ---- serialise
        // boxes round outward by one float step: every primitive stays inside
        // its float box whatever the rounding of its own vertices
        auto fbox = [](const Box& b, int i, bool hi) {
            return hi ? std::nextafter((float)b.hi[i], INFINITY) : std::nextafter((float)b.lo[i], -INFINITY);
        };
        auto aux_of = [&](int ni, int ch) {
            if (which == 1) return make_float4((float)sub_meas[ni * 2 + ch], 0.f, 0.f, 0.f);
            if (which == 2) {
                // normal cone as (axis, cos of the half-angle); cos <= 0 marks
                // a cone that never culls (half-angle >= pi/2, an undefined
                // axis, or a subtree holding a boundary feature).  The cosine
                // is rounded down so the stored cone contains the exact one.
                auto& c = sub_cone[ni * 2 + ch];
                const bool off = brute || sub_bnd[ni * 2 + ch] || !(c[3] > 0.0);
                const float cw = off ? -1.f : std::nextafter((float)c[3], -INFINITY);
                return make_float4((float)c[0], (float)c[1], (float)c[2], cw);
            }
            return make_float4(0.f, 0.f, 0.f, 0.f);
        };
        // ---- collapse into four-wide nodes: a node holds the children of a
        // binary node, with every inner child replaced by its own two
        // children (breadth first, so every inner reference points forward)
        struct Ent { int bn, ch; };                 // child `ch` of binary node `bn`
        std::vector<std::array<Ent, 4>> ent4;
        std::vector<int> n_ent4, depth4;
        std::vector<int> of_binary(nn, -1);         // binary node -> four-wide node
        int max_d4 = 0;
        if (nn > 0) {
            std::vector<int> queue{0};
            of_binary[0] = 0;
            ent4.emplace_back();
            n_ent4.push_back(0);
            depth4.push_back(1);
            for (size_t qi = 0; qi < queue.size(); ++qi) {
                const int bn = queue[qi];
                const int me = of_binary[bn];
                max_d4 = std::max(max_d4, depth4[me]);
                std::array<Ent, 4> e{};
                int m = 0;
                const BuiltNode& nd = B.nodes[bn];
                for (int ch = 0; ch < 2; ++ch) {
                    if (nd.n[ch] > 0) { e[m++] = {bn, ch}; continue; }
                    if (nd.c[ch] < 0) continue;
                    const BuiltNode& cd = B.nodes[nd.c[ch]];
                    for (int gch = 0; gch < 2; ++gch)
                        if (cd.n[gch] > 0 || cd.c[gch] >= 0) e[m++] = {nd.c[ch], gch};
                }
                for (int k = 0; k < m; ++k) {
                    const BuiltNode& pn = B.nodes[e[k].bn];
                    if (pn.n[e[k].ch] > 0) continue;
                    const int child = pn.c[e[k].ch];
                    of_binary[child] = (int)ent4.size();
                    ent4.emplace_back();
                    n_ent4.push_back(0);
                    depth4.push_back(depth4[me] + 1);
                    queue.push_back(child);
                }
                ent4[me] = e;
                n_ent4[me] = m;
            }
        }
        const int n4 = (int)ent4.size();
        // a lane defers at most three children per level of its path
        const int stack_need = 3 * std::max(max_d4 - 1, 0) + 1;
        g->stack_entries = std::max(g->stack_entries, stack_need);
        if (stack_need > kMaxStack || (int64_t)np > kMaxLeafFirst || leaf > kLeafMax) {
            set_error("wost_build_bvh: hierarchy %d too deep or too large (stack %d > %d or %d primitives)", which,
                      stack_need, kMaxStack, np);
            delete g;
            return WOST_EUNSUPPORTED;
        }
        const int stride = which == 0 ? 2 * d + 1 : which == 1 ? 2 * d + 2 : 3 * d + 3;
        const Box all_box = B.range_box(0, (int)items.size());
        std::vector<float4> nodes4((size_t)n4 * stride);
        for (int i = 0; i < n4; ++i) {
            float lo[3][4], hi[3][4], aux[4][4];
            int32_t ref[4], pcs[4] = {-1, -1, -1, -1};
            for (int k = 0; k < 4; ++k) {
                for (int a = 0; a < 3; ++a) { lo[a][k] = INFINITY; hi[a][k] = -INFINITY; }
                for (int a = 0; a < 4; ++a) aux[a][k] = 0.f;
                ref[k] = kEmptyRef;
                if (k >= n_ent4[i]) continue;
                const Ent en = ent4[i][k];
                const BuiltNode& pn = B.nodes[en.bn];
                const Box& cb = brute ? all_box : pn.box[en.ch];
                for (int a = 0; a < d; ++a) { lo[a][k] = fbox(cb, a, 0); hi[a][k] = fbox(cb, a, 1); }
                ref[k] = pn.n[en.ch] > 0 ? leaf_ref(pn.c[en.ch], pn.n[en.ch]) : of_binary[pn.c[en.ch]];
                const float4 ax = aux_of(en.bn, en.ch);
                if (which == 1) aux[0][k] = ax.x;
                if (which == 2) {
                    const float v[4] = {ax.x, ax.y, ax.z, ax.w};
                    for (int a = 0; a < d; ++a) aux[a][k] = v[a];
                    aux[d][k] = v[3];
                    pcs[k] = brute ? -1 : sub_piece[en.bn * 2 + en.ch];
                }
            }
            float4* o = &nodes4[(size_t)i * stride];
            for (int a = 0; a < d; ++a) {
                o[a] = make_float4(lo[a][0], lo[a][1], lo[a][2], lo[a][3]);
                o[d + a] = make_float4(hi[a][0], hi[a][1], hi[a][2], hi[a][3]);
            }
            int4 r = make_int4(ref[0], ref[1], ref[2], ref[3]);
            memcpy(&o[2 * d], &r, sizeof(r));
            const int n_aux = which == 1 ? 1 : which == 2 ? d + 1 : 0;
            for (int a = 0; a < n_aux; ++a) o[2 * d + 1 + a] = make_float4(aux[a][0], aux[a][1], aux[a][2], aux[a][3]);
            if (which == 2) {
                const int4 pv = make_int4(pcs[0], pcs[1], pcs[2], pcs[3]);
                memcpy(&o[3 * d + 2], &pv, sizeof(pv));
            }
        }
        // validation of the four-wide references (the kernels index without checks)
        {
            std::vector<int> seen(np, 0);
            bool ok = (n4 > 0) == (np > 0);
            for (int i = 0; i < n4 && ok; ++i) {
                int32_t r[4];
                memcpy(r, &nodes4[(size_t)i * stride + 2 * d], sizeof(r));
                for (int k = 0; k < 4 && ok; ++k) {
                    if (r[k] == kEmptyRef) continue;
                    if (r[k] >= 0) { ok = r[k] > i && r[k] < n4; continue; }
                    const int f = leaf_first(r[k]), c = leaf_count(r[k]);
                    ok = f >= 0 && c >= 1 && f + c <= np;
                    for (int j = f; ok && j < f + c; ++j) seen[j]++;
                }
            }
            for (int j = 0; j < np && ok; ++j) ok = seen[j] == 1;
            if (!ok) {
                set_error("wost_build_bvh: internal error: four-wide hierarchy %d failed validation", which);
                delete g;
                return WOST_EINVAL;
            }
        }
        const int64_t off_nodes = push_bytes(img, nodes4.data(), nodes4.size());
        std::vector<float4> pr;
        std::vector<float4> px;
        std::vector<int32_t> orig;
        for (int k = 0; k < np; ++k) {
            int32_t id = B.order[k];
            if (which < 2) {
                const double* a = &P[(size_t)id * d * d];
                if (d == 2) {
                    pr.push_back(make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]));
                } else {
                    // the three vertices as given (rounded once to float), so
                    // triangles sharing an edge hold bit-identical endpoints
                    pr.push_back(make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]));
                    pr.push_back(make_float4((float)a[4], (float)a[5], (float)a[6], (float)a[7]));
                    pr.push_back(make_float4((float)a[8], 0.f, 0.f, 0.f));
                }
                if (which == 1)
                    px.push_back(make_float4((float)nout[id][0], (float)nout[id][1], (float)nout[id][2], (float)meas[id]));
                orig.push_back(id);
            } else {
                const Sil& s = sils[id];
                if (d == 2) {
                    // adjacent primitives as internal Neumann ids (float bit patterns)
                    const float f1 = int_bits(neu_internal[s.q1]);
                    const float f2 = int_bits(s.q2 >= 0 ? neu_internal[s.q2] : -1);
                    pr.push_back(make_float4((float)s.a[0], (float)s.a[1], (float)s.n1[0], (float)s.n1[1]));
                    pr.push_back(make_float4((float)s.n2[0], (float)s.n2[1], f1, f2));
                } else {
                    const float f1 = int_bits(neu_internal[s.q1]);
                    const float f2 = int_bits(s.q2 >= 0 ? neu_internal[s.q2] : -1);
                    pr.push_back(make_float4((float)s.a[0], (float)s.a[1], (float)s.a[2], (float)s.b[0]));
                    pr.push_back(make_float4((float)s.b[1], (float)s.b[2], (float)s.n1[0], (float)s.n1[1]));
                    pr.push_back(make_float4((float)s.n1[2], (float)s.n2[0], (float)s.n2[1], (float)s.n2[2]));
                    pr.push_back(make_float4(f1, f2, 0.f, 0.f));
                }
            }
        }
        int64_t off_prims = push_bytes(img, pr.data(), pr.size());
        int64_t off_px = which == 1 ? push_bytes(img, px.data(), px.size()) : -1;
        int64_t off_orig = which < 2 ? push_bytes(img, orig.data(), orig.size()) : -1;
        int64_t off_piece = -1;
        if (which == 2) {
            // convex piece of every Neumann primitive, by internal id
            std::vector<int32_t> pc(std::max<int64_t>(g->n_neu, 1), -1);
            for (int64_t q = 0; q < n_prims; ++q)
                if (bc[q] && neu_internal[q] >= 0) pc[neu_internal[q]] = brute ? -1 : seg_piece[q];
            off_piece = push_bytes(img, pc.data(), pc.size());
        }
        g->sec[which] = {off_nodes, off_prims, off_px, off_orig, off_piece, n4, np};
        if (which == 0) g->n_dir = np;
        if (which == 1) {
            g->n_neu = np;
            for (int k = 0; k < np; ++k) neu_internal[B.order[k]] = k;
        }
        if (which == 2) g->n_sil = np;
        if (which < 2) orig_all.insert(orig_all.end(), orig.begin(), orig.end());
    }
    g->off_neu_id = push_bytes(img, neu_internal.data(), neu_internal.size());
    g->n_caller = n_prims;
    img.resize((img.size() + 255) & ~size_t(255));
    g->bytes = (int64_t)img.size();
    g->image = (uint8_t*)malloc(img.size());
    memcpy(g->image, img.data(), img.size());
    g->orig_host = (int32_t*)malloc(sizeof(int32_t) * (orig_all.size() + 1));
    memcpy(g->orig_host, orig_all.data(), sizeof(int32_t) * orig_all.size());
    *out = g;
    return WOST_OK;
}

extern "C" int64_t wost_geom_device_bytes(const wost_geom* g) { return g ? g->bytes : -1; }

extern "C" int wost_geom_upload(wost_geom* g, void* dev_buf, int64_t bytes, void* stream)
{
    if (!g || !dev_buf) { set_error("wost_geom_upload: NULL argument"); return WOST_EINVAL; }
    if (bytes < g->bytes) { set_error("wost_geom_upload: buffer has %lld bytes, need %lld", (long long)bytes, (long long)g->bytes); return WOST_ESIZE; }
    if (((uintptr_t)dev_buf) & 255) { set_error("wost_geom_upload: buffer must be 256-byte aligned"); return WOST_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (g->image) {
        e = hipMemcpyAsync(dev_buf, g->image, g->bytes, hipMemcpyHostToDevice, s);
    } else {
        // device-built: padding zeroed as in the host image, then every array
        e = hipMemsetAsync(dev_buf, 0, g->bytes, s);
        for (size_t k = 0; k < g->staged.size() && e == hipSuccess; ++k)
            e = hipMemcpyAsync((uint8_t*)dev_buf + g->staged[k].off, g->staged[k].src, g->staged[k].bytes,
                               hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_error("wost_geom_upload: %s", hipGetErrorString(e)); return WOST_EHIP; }
    g->dev = dev_buf;
    return WOST_OK;
}

extern "C" int wost_geom_info(const wost_geom* g, double* o)
{
    if (!g || !o) { set_error("wost_geom_info: NULL argument"); return WOST_EINVAL; }
    o[0] = g->dim; o[1] = (double)g->n_dir; o[2] = (double)g->n_neu; o[3] = (double)g->n_sil;
    o[4] = g->max_depth; o[5] = g->diag; o[6] = (double)g->bytes; o[7] = g->stack_entries;
    return WOST_OK;
}

extern "C" int64_t wost_geom_prim_index(const wost_geom* g, int32_t internal_id)
{
    if (!g || internal_id < 0 || internal_id >= g->n_dir + g->n_neu) return -1;
    return g->orig_host[internal_id];
}

extern "C" void wost_geom_free(wost_geom* g)
{
    if (!g) return;
    free(g->image);
    free(g->orig_host);
    delete g;
}
