// The geometry image built on the GPU from device inputs: the Dirichlet
// hierarchy, the Neumann hierarchy with subtree measures (area sampling of
// the Neumann term, Sec. 4.2) and the silhouette-candidate hierarchy with
// normal cones and 2D convex pieces (closest silhouette point, Sec. 3.2 and
// the query library of Sec. 5.3), byte for byte the image that the host
// builder writes for the same input.
//
// Every number is computed with the host builder's floating-point operations
// (FP64 where it uses FP64; products are never fused into multiply-adds in
// this file), and every choice the host makes by order is made here by the
// same rule:
//  * per primitive: outward normal and measure, input validation;
//  * classes: a stable radix sort of the caller indices by condition;
//  * silhouette candidates: vertex keys (2D) or (smaller, larger) vertex
//    pairs of edges (3D) of the Neumann primitives, stably sorted; a run of
//    equal keys is one candidate whose neighbours are its first two entries;
//  * 2D convex pieces: links at strictly convex vertices whose segments run
//    the same way with normals in one quadrant, named by pointer jumping;
//  * a hierarchy: median splits level by level.  Each item has a rank per
//    axis (its position in the order of centroid coordinate, then index);
//    a level sorts every open range by its longest centroid axis' rank with
//    two stable passes (rank, then range), halves it, and numbers the inner
//    children in the host's depth-first preorder, which follows from subtree
//    sizes alone.  Leaves list their items by index;
//  * per-child aggregates bottom-up level by level in the host's order of
//    summation; cone half-angles from exact atomic minima of cosines;
//  * the four-wide collapse breadth first, node indices from prefix sums.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "radix_sort.h"
#include "wost_internal.h"

#pragma clang fp contract(off)

namespace wost {
namespace {

constexpr int kT = 256;

inline int blocks(int64_t n) { return (int)std::max<int64_t>((n + kT - 1) / kT, 1); }
inline int bits_for(int64_t n)
{
    int b = 1;
    while (b < 32 && (int64_t(1) << b) < n) ++b;
    return b;
}

// order-preserving integer images of floats and doubles (negative zero taken
// as zero), so that exact minima and maxima can be taken with integer atomics
__device__ __forceinline__ uint32_t f_ord(float x)
{
    const uint32_t u = __float_as_uint(x + 0.0f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float f_unord(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}
__device__ __forceinline__ uint64_t d_ord(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x + 0.0);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double d_unord(uint64_t u)
{
    return __longlong_as_double((long long)((u >> 63) ? (u & ~(1ull << 63)) : ~u));
}
// the neighbouring float toward -inf / +inf (finite x)
__device__ __forceinline__ float f_down(float x)
{
    const uint32_t u = __float_as_uint(x);
    if (x == 0.f) return __uint_as_float(0x80000001u);
    return __uint_as_float(x > 0.f ? u - 1u : u + 1u);
}
__device__ __forceinline__ float f_up(float x)
{
    const uint32_t u = __float_as_uint(x);
    if (x == 0.f) return __uint_as_float(0x00000001u);
    return __uint_as_float(x > 0.f ? u + 1u : u - 1u);
}

// inner nodes of a median-split subtree over s items with leaves of at most
// L items: the sizes on one level are two consecutive values, so count level
// by level how many subtrees of each size split
__host__ __device__ inline int64_t inner_count(int64_t s, int L)
{
    int64_t lo = s, n_lo = 1, n_hi = 0, total = 0;
    for (;;) {
        const int64_t in_lo = lo > L ? n_lo : 0, in_hi = lo + 1 > L ? n_hi : 0;
        if (in_lo + in_hi == 0) return total;
        total += in_lo + in_hi;
        const int64_t h = lo / 2;
        int64_t c_h = 0, c_h1 = 0;
        // size x splits into x / 2 and x - x / 2
        if (lo % 2 == 0) c_h += 2 * in_lo;
        else { c_h += in_lo; c_h1 += in_lo; }
        if ((lo + 1) % 2 == 0) c_h1 += 2 * in_hi;
        else { c_h += in_hi; c_h1 += in_hi; }
        lo = h;
        n_lo = c_h;
        n_hi = c_h1;
    }
}

// smallest (stage, index, kind) error: the host reports the first in its
// loop order (vertices, then primitives)
__device__ __forceinline__ void report(unsigned long long* err, int stage, int64_t index, int kind)
{
    atomicMin(err, ((unsigned long long)stage << 60) | ((unsigned long long)index << 4) | (unsigned long long)kind);
}

// ------------------------------------------------------------ primitives

template <int D>
__global__ __launch_bounds__(kT) void gb_verts(const float* verts, int64_t V, uint32_t* vb, unsigned long long* err)
{
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= V) return;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float x = verts[v * D + a];
        if (!isfinite(x)) { report(err, 0, v, 0); return; }
        atomicMin(&vb[a], f_ord(x));
        atomicMax(&vb[3 + a], f_ord(x));
    }
}

// outward normal and measure in FP64, validation, and the Neumann count
template <int D>
__global__ __launch_bounds__(kT) void gb_prims(const float* verts, int64_t V, const int32_t* prims, int P,
                                               const uint8_t* bc, double* nout, double* meas, uint32_t* counters,
                                               unsigned long long* err)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q >= P) return;
    if (bc[q] > 1) { report(err, 1, q, 1); return; }
    double a[D][D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int32_t vid = prims[(int64_t)q * D + k];
        if (vid < 0 || vid >= V) { report(err, 1, q, 2); return; }
#pragma unroll
        for (int i = 0; i < D; ++i) a[k][i] = (double)verts[(int64_t)vid * D + i];
    }
    if (D == 2) {
        const double ex = a[1][0] - a[0][0], ey = a[1][1] - a[0][1];
        const double len = sqrt(ex * ex + ey * ey);
        if (!(len > 0)) { report(err, 1, q, 3); return; }
        nout[(int64_t)q * 3] = ey / len;
        nout[(int64_t)q * 3 + 1] = -ex / len;
        nout[(int64_t)q * 3 + 2] = 0.0;
        meas[q] = len;
    } else {
        double e1[3], e2[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) { e1[i] = a[1][i % D] - a[0][i % D]; e2[i] = a[D - 1][i % D] - a[0][i % D]; }
        const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!(len > 0)) { report(err, 1, q, 4); return; }
        nout[(int64_t)q * 3] = c[0] / len;
        nout[(int64_t)q * 3 + 1] = c[1] / len;
        nout[(int64_t)q * 3 + 2] = c[2] / len;
        meas[q] = 0.5 * len;
    }
    if (bc[q]) atomicAdd(&counters[0], 1u);
}

__global__ __launch_bounds__(kT) void gb_class_keys(const uint8_t* bc, int P, uint32_t* keys, int32_t* vals)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q >= P) return;
    keys[q] = bc[q];
    vals[q] = q;
}

// items of a primitive hierarchy: float box of the vertices, FP64 centroid
template <int D>
__global__ __launch_bounds__(kT) void gb_items_prims(const float* verts, const int32_t* prims, const int32_t* list,
                                                     int m, int ms, float* blo, float* bhi, double* cen)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    const int q = list[i];
    float lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int32_t vid = prims[(int64_t)q * D + k];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const float x = verts[(int64_t)vid * D + a];
            lo[a] = k == 0 ? x : fminf(lo[a], x);
            hi[a] = k == 0 ? x : fmaxf(hi[a], x);
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        blo[(int64_t)a * ms + i] = lo[a];
        bhi[(int64_t)a * ms + i] = hi[a];
        cen[(int64_t)a * ms + i] = 0.5 * ((double)lo[a] + (double)hi[a]);
    }
}

// ------------------------------------------------------------ hierarchy

__global__ __launch_bounds__(kT) void gb_iota(int32_t* a, int m)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i < m) a[i] = i;
}

__global__ __launch_bounds__(kT) void gb_copy_i32(const int32_t* src, int32_t* dst, int m)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i < m) dst[i] = src[i];
}

__global__ __launch_bounds__(kT) void gb_fill_u32(uint32_t* a, int64_t m, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) a[i] = v;
}

__global__ __launch_bounds__(kT) void gb_fill_i32(int32_t* a, int64_t m, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) a[i] = v;
}

// rank keys: the low, then the high half of the ordered image of the centroid
__global__ __launch_bounds__(kT) void gb_rank_lo(const double* c, int m, uint32_t* keys, int32_t* vals)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    keys[i] = (uint32_t)d_ord(c[i]);
    vals[i] = i;
}

__global__ __launch_bounds__(kT) void gb_rank_hi(const double* c, const int32_t* sorted, int m, uint32_t* keys,
                                                 int32_t* vals)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    const int i = sorted[p];
    keys[p] = (uint32_t)(d_ord(c[i]) >> 32);
    vals[p] = i;
}

__global__ __launch_bounds__(kT) void gb_rank_store(const int32_t* sorted, int m, uint32_t* rank)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p < m) rank[sorted[p]] = (uint32_t)p;
}

// open range of every position (binary search over the level's ranges,
// which are sorted by position) and the key that keeps ranges and the gaps
// between them in place in the stable sort by range
__global__ __launch_bounds__(kT) void gb_level_pos(int m, const int32_t* rb, const int32_t* re, int R,
                                                   const int32_t* perm, int32_t* pslot, uint32_t* key2)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    int lo = 0, hi = R - 1, s = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (rb[mid] <= p) { s = mid; lo = mid + 1; }
        else hi = mid - 1;
    }
    const bool open = s >= 0 && p < re[s];
    pslot[p] = open ? s : -1;
    key2[perm[p]] = open ? 2u * (uint32_t)s + 1u : 2u * (uint32_t)(s + 1);
}

template <int D>
__global__ __launch_bounds__(kT) void gb_cbox_init(uint64_t* cbox, int R)
{
    const int s = blockIdx.x * kT + threadIdx.x;
    if (s >= R) return;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        cbox[(int64_t)s * 2 * D + a] = ~0ull;
        cbox[(int64_t)s * 2 * D + D + a] = 0ull;
    }
}

// centroid bounds of every open range: exact minima and maxima; a wave whose
// lanes all fall in one range reduces before its single atomic
template <int D>
__global__ __launch_bounds__(kT) void gb_cbox(int m, const int32_t* pslot, const int32_t* perm, const double* cen,
                                              int ms, uint64_t* cbox)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    const int s = p < m ? pslot[p] : -1;
    const int s0 = __shfl(s, 0);
    const bool uniform = __all(s == s0) && s0 >= 0;
    if (!uniform && s < 0) return;
    const int item = s >= 0 ? perm[p] : 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        uint64_t v = s >= 0 ? d_ord(cen[(int64_t)a * ms + item]) : 0ull;
        if (uniform) {
            uint64_t lo = v, hi = v;
            for (int o = 32; o > 0; o >>= 1) {
                const uint64_t l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
                lo = l2 < lo ? l2 : lo;
                hi = h2 > hi ? h2 : hi;
            }
            if ((threadIdx.x & 63) == 0) {
                atomicMin((unsigned long long*)&cbox[(int64_t)s0 * 2 * D + a], (unsigned long long)lo);
                atomicMax((unsigned long long*)&cbox[(int64_t)s0 * 2 * D + D + a], (unsigned long long)hi);
            }
        } else {
            atomicMin((unsigned long long*)&cbox[(int64_t)s * 2 * D + a], (unsigned long long)v);
            atomicMax((unsigned long long*)&cbox[(int64_t)s * 2 * D + D + a], (unsigned long long)v);
        }
    }
}

// split axis: the longest centroid extent, the first on ties
template <int D>
__global__ __launch_bounds__(kT) void gb_axis(int R, const uint64_t* cbox, int32_t* rax)
{
    const int s = blockIdx.x * kT + threadIdx.x;
    if (s >= R) return;
    double ext[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
        ext[a] = d_unord(cbox[(int64_t)s * 2 * D + D + a]) - d_unord(cbox[(int64_t)s * 2 * D + a]);
    int ax = 0;
#pragma unroll
    for (int a = 1; a < D; ++a)
        if (ext[a] > ext[ax]) ax = a;
    rax[s] = ax;
}

__global__ __launch_bounds__(kT) void gb_level_keys(int m, const int32_t* pslot, const int32_t* perm,
                                                    const int32_t* rax, const uint32_t* rank, int ms, uint32_t* keys,
                                                    int32_t* vals)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    const int s = pslot[p], item = perm[p];
    keys[p] = s >= 0 ? rank[(int64_t)rax[s] * ms + item] : 0u;
    vals[p] = item;
}

__global__ __launch_bounds__(kT) void gb_level_keys2(int m, const int32_t* sorted, const uint32_t* key2,
                                                     uint32_t* keys, int32_t* vals)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    const int item = sorted[p];
    keys[p] = key2[item];
    vals[p] = item;
}

struct TreeBufs {
    int32_t* nc;        // [2 nn] child: first leaf position (leaf) or node index (inner), -1 empty
    int32_t* ncount;    // [2 nn] leaf item count, 0 for inner or empty children
    int32_t* parent;    // [nn] parent child slot (2 node + side), -1 at the root
    uint32_t* nbox;     // [2 nn][6] ordered child boxes: lo xyz, hi xyz
    int32_t* leaves;    // [3 * leaves] first, count, child slot
    int32_t* pleaf;     // [m] child slot of the leaf holding each position
    uint32_t* counters; // [0] leaves, [1] deepest leaf, [2] scan total
};

__device__ __forceinline__ void make_leaf(const TreeBufs& t, int slot, int first, int n, int depth)
{
    t.nc[slot] = first;
    t.ncount[slot] = n;
    const int li = (int)atomicAdd(&t.counters[0], 1u);
    t.leaves[3 * li] = first;
    t.leaves[3 * li + 1] = n;
    t.leaves[3 * li + 2] = slot;
    for (int p = first; p < first + n; ++p) t.pleaf[p] = slot;
    atomicMax(&t.counters[1], (uint32_t)depth);
}

// halves every open range: leaf children are recorded, inner children get
// their preorder index (left: the next index; right: after the left subtree)
__global__ __launch_bounds__(kT) void gb_children(int R, const int32_t* rb, const int32_t* re, const int32_t* rnode,
                                                  int L, int depth, TreeBufs t, uint32_t* open_count)
{
    const int s = blockIdx.x * kT + threadIdx.x;
    if (s >= R) return;
    const int b = rb[s], e = re[s], nd = rnode[s];
    const int mid = b + (e - b) / 2;
    const int ls = mid - b, rs = e - mid;
    uint32_t open = 0;
    if (ls <= L) make_leaf(t, 2 * nd, b, ls, depth + 1);
    else { t.nc[2 * nd] = nd + 1; t.ncount[2 * nd] = 0; t.parent[nd + 1] = 2 * nd; ++open; }
    const int ri = nd + 1 + (int)inner_count(ls, L);
    if (rs <= L) make_leaf(t, 2 * nd + 1, mid, rs, depth + 1);
    else { t.nc[2 * nd + 1] = ri; t.ncount[2 * nd + 1] = 0; t.parent[ri] = 2 * nd + 1; ++open; }
    open_count[s] = open;
}

template <int D>
__global__ __launch_bounds__(kT) void gb_child_boxes(int m, const int32_t* pslot, const int32_t* rb,
                                                     const int32_t* re, const int32_t* rnode, const int32_t* perm,
                                                     const float* blo, const float* bhi, int ms, uint32_t* nbox)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    const int s = p < m ? pslot[p] : -1;
    int slot = -1;
    if (s >= 0) slot = 2 * rnode[s] + (p >= rb[s] + (re[s] - rb[s]) / 2 ? 1 : 0);
    const int s0 = __shfl(slot, 0);
    const bool uniform = __all(slot == s0) && s0 >= 0;
    if (!uniform && slot < 0) return;
    const int item = slot >= 0 ? perm[p] : 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        uint32_t lo = slot >= 0 ? f_ord(blo[(int64_t)a * ms + item]) : ~0u;
        uint32_t hi = slot >= 0 ? f_ord(bhi[(int64_t)a * ms + item]) : 0u;
        if (uniform) {
            for (int o = 32; o > 0; o >>= 1) {
                lo = min(lo, (uint32_t)__shfl_xor(lo, o));
                hi = max(hi, (uint32_t)__shfl_xor(hi, o));
            }
            if ((threadIdx.x & 63) == 0) {
                atomicMin(&nbox[(int64_t)s0 * 6 + a], lo);
                atomicMax(&nbox[(int64_t)s0 * 6 + 3 + a], hi);
            }
        } else {
            atomicMin(&nbox[(int64_t)slot * 6 + a], lo);
            atomicMax(&nbox[(int64_t)slot * 6 + 3 + a], hi);
        }
    }
}

__global__ __launch_bounds__(kT) void gb_box_init(uint32_t* nbox, int64_t slots)
{
    const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (k >= slots) return;
    for (int a = 0; a < 3; ++a) { nbox[k * 6 + a] = ~0u; nbox[k * 6 + 3 + a] = 0u; }
}

__global__ __launch_bounds__(kT) void gb_next_ranges(int R, const int32_t* rb, const int32_t* re,
                                                     const int32_t* rnode, int L, const uint32_t* offs, int32_t* nb,
                                                     int32_t* ne, int32_t* nnode, int32_t* lvl)
{
    const int s = blockIdx.x * kT + threadIdx.x;
    if (s >= R) return;
    const int b = rb[s], e = re[s], nd = rnode[s];
    const int mid = b + (e - b) / 2;
    const int ls = mid - b, rs = e - mid;
    int k = (int)offs[s];
    if (ls > L) { nb[k] = b; ne[k] = mid; nnode[k] = nd + 1; lvl[k] = nd + 1; ++k; }
    if (rs > L) {
        const int ri = nd + 1 + (int)inner_count(ls, L);
        nb[k] = mid; ne[k] = e; nnode[k] = ri; lvl[k] = ri;
    }
}

// a hierarchy of at most L items: the root holds one leaf child
__global__ void gb_root_leaf(int m, TreeBufs t)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    t.nc[1] = -1;
    t.ncount[1] = 0;
    t.parent[0] = -1;
    make_leaf(t, 0, 0, m, 1);
}

template <int D>
__global__ __launch_bounds__(kT) void gb_root_box(int m, const float* blo, const float* bhi, int ms, uint32_t* nbox)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        atomicMin(&nbox[a], f_ord(blo[(int64_t)a * ms + i]));
        atomicMax(&nbox[3 + a], f_ord(bhi[(int64_t)a * ms + i]));
    }
}

// a leaf's items by index (at most 64: insertion sort by one thread)
__global__ __launch_bounds__(kT) void gb_leaf_sort(int n_leaves, const int32_t* leaves, int32_t* perm)
{
    const int l = blockIdx.x * kT + threadIdx.x;
    if (l >= n_leaves) return;
    int32_t* p = perm + leaves[3 * l];
    const int n = leaves[3 * l + 1];
    for (int i = 1; i < n; ++i) {
        const int32_t v = p[i];
        int j = i - 1;
        while (j >= 0 && p[j] > v) { p[j + 1] = p[j]; --j; }
        p[j + 1] = v;
    }
}

// ------------------------------------------------------------ aggregates

__global__ __launch_bounds__(kT) void gb_gather_meas(const int32_t* list, int m, const double* meas, double* out)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i < m) out[i] = meas[list[i]];
}

// Neumann: measure of every child, summed in leaf order; a node adds its two
// children's measures
__global__ __launch_bounds__(kT) void gb_agg_neu(const int32_t* lvl, int count, const TreeBufs t, const int32_t* perm,
                                                 const double* imeas, double* sub_meas, double* node_meas)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= count) return;
    const int nd = lvl[i];
    double nm = 0.0;
    for (int ch = 0; ch < 2; ++ch) {
        const int k2 = 2 * nd + ch, c = t.nc[k2], n = t.ncount[k2];
        double m = 0.0;
        if (n > 0) {
            for (int p = c; p < c + n; ++p) m += imeas[perm[p]];
        } else if (c >= 0) {
            m = node_meas[c];
        }
        sub_meas[k2] = m;
        nm += m;
    }
    node_meas[nd] = nm;
}

struct SilAgg {
    double* sub_sum;    // [2 nn][3]
    double* node_sum;   // [nn][3]
    int32_t* sub_cnt;   // [2 nn] normals below
    int32_t* node_cnt;
    int32_t* sub_bnd;   // [2 nn] a boundary feature below
    int32_t* node_bnd;
    int32_t* sub_piece; // [2 nn] the piece all candidates below share, or -1
    int32_t* node_piece;
    double* axis;       // [2 nn][3] normalised sum; (1, 0, 0) when undefined
    int32_t* valid;     // [2 nn] the axis is defined
    uint64_t* worst;    // [2 nn] ordered smallest cosine to the axis
};

struct SilItems {
    const double* n1;   // [C][3] inward normals of the neighbours
    const double* n2;
    const int32_t* bnd; // [C] single Neumann neighbour
    const int32_t* piece;
};

__device__ __forceinline__ int32_t join_piece(int32_t a, int32_t b)
{
    return a == -2 ? b : (b == -2 ? a : (a == b ? a : -1));
}

__global__ __launch_bounds__(kT) void gb_agg_sil(const int32_t* lvl, int count, const TreeBufs t, const int32_t* perm,
                                                 const SilItems it, SilAgg g)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= count) return;
    const int nd = lvl[i];
    double nsum[3] = {0.0, 0.0, 0.0};
    int32_t ncnt = 0, nbnd = 0, npc = -2;
    for (int ch = 0; ch < 2; ++ch) {
        const int k2 = 2 * nd + ch, c = t.nc[k2], n = t.ncount[k2];
        double s[3] = {0.0, 0.0, 0.0};
        int32_t cnt = 0, bnd = 0, pc = -2;
        if (n > 0) {
            for (int p = c; p < c + n; ++p) {
                const int k = perm[p];
                for (int a = 0; a < 3; ++a) s[a] += it.n1[(int64_t)k * 3 + a];
                ++cnt;
                if (!it.bnd[k]) {
                    for (int a = 0; a < 3; ++a) s[a] += it.n2[(int64_t)k * 3 + a];
                    ++cnt;
                }
                bnd = bnd || it.bnd[k];
                pc = join_piece(pc, it.piece[k]);
            }
        } else if (c >= 0) {
            for (int a = 0; a < 3; ++a) s[a] = g.node_sum[(int64_t)c * 3 + a];
            cnt = g.node_cnt[c];
            bnd = g.node_bnd[c];
            pc = g.node_piece[c];
        }
        for (int a = 0; a < 3; ++a) { g.sub_sum[(int64_t)k2 * 3 + a] = s[a]; nsum[a] += s[a]; }
        g.sub_cnt[k2] = cnt;
        g.sub_bnd[k2] = bnd;
        g.sub_piece[k2] = pc == -2 ? -1 : pc;
        ncnt += cnt;
        nbnd = nbnd || bnd;
        npc = join_piece(npc, pc);
    }
    for (int a = 0; a < 3; ++a) g.node_sum[(int64_t)nd * 3 + a] = nsum[a];
    g.node_cnt[nd] = ncnt;
    g.node_bnd[nd] = nbnd;
    g.node_piece[nd] = npc == -2 ? -1 : npc;
}

__global__ __launch_bounds__(kT) void gb_axes(int slots, SilAgg g)
{
    const int k2 = blockIdx.x * kT + threadIdx.x;
    if (k2 >= slots) return;
    const double* s = g.sub_sum + (int64_t)k2 * 3;
    const double len = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    const int cnt = g.sub_cnt[k2];
    const bool ok = !(cnt == 0 || len < 1e-9 * (double)cnt);
    g.axis[(int64_t)k2 * 3] = ok ? s[0] / len : 1.0;
    g.axis[(int64_t)k2 * 3 + 1] = ok ? s[1] / len : 0.0;
    g.axis[(int64_t)k2 * 3 + 2] = ok ? s[2] / len : 0.0;
    g.valid[k2] = ok;
    g.worst[k2] = d_ord(ok ? 1.0 : -1.0);
}

// every candidate lowers the cosine bound of each child on its path to the root
__global__ __launch_bounds__(kT) void gb_worst(int m, const int32_t* perm, const TreeBufs t, const SilItems it,
                                               SilAgg g)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    const int k = perm[p];
    const double* n1 = it.n1 + (int64_t)k * 3;
    const double* n2 = it.n2 + (int64_t)k * 3;
    const bool two = !it.bnd[k];
    int slot = t.pleaf[p];
    // a path is at most 62 splits long (the build stops deeper trees)
    for (int up = 0; up < 64; ++up) {
        if (g.valid[slot]) {
            const double* ax = g.axis + (int64_t)slot * 3;
            double w = ax[0] * n1[0] + ax[1] * n1[1] + ax[2] * n1[2];
            if (two) {
                const double w2 = ax[0] * n2[0] + ax[1] * n2[1] + ax[2] * n2[2];
                w = w2 < w ? w2 : w;
            }
            atomicMin((unsigned long long*)&g.worst[slot], (unsigned long long)d_ord(w));
        }
        const int nd = slot >> 1;
        if (nd == 0) break;
        slot = t.parent[nd];
    }
}

// ------------------------------------------------------------ four-wide collapse

// the children of binary node bn with every inner child replaced by its own
// non-empty children: up to four child slots (2 node + side)
__device__ __forceinline__ int entries_of(int bn, const TreeBufs& t, int e[4])
{
    int n = 0;
    for (int ch = 0; ch < 2; ++ch) {
        const int k2 = 2 * bn + ch;
        if (t.ncount[k2] > 0) { e[n++] = k2; continue; }
        const int c = t.nc[k2];
        if (c < 0) continue;
        for (int g = 0; g < 2; ++g)
            if (t.ncount[2 * c + g] > 0 || t.nc[2 * c + g] >= 0) e[n++] = 2 * c + g;
    }
    return n;
}

__global__ __launch_bounds__(kT) void gb_c4_count(int Q, const int32_t* qbn, const TreeBufs t, uint32_t* cnt)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= Q) return;
    int e[4];
    const int n = entries_of(qbn[i], t, e);
    uint32_t c = 0;
    for (int k = 0; k < n; ++k) c += t.ncount[e[k]] == 0;
    cnt[i] = c;
}

struct C4Aux {
    const double* sub_meas;     // Neumann
    const double* axis;         // silhouettes
    const int32_t* valid;
    const uint64_t* worst;
    const int32_t* sub_bnd;
    const int32_t* sub_piece;
};

// KIND 0 Dirichlet, 1 Neumann, 2 silhouettes
template <int D, int KIND>
__global__ __launch_bounds__(kT) void gb_c4_write(int Q, const int32_t* qbn, const int32_t* qme, const uint32_t* offs,
                                                  int base, const TreeBufs t, const C4Aux x, float4* nodes,
                                                  int32_t* nqbn, int32_t* nqme)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= Q) return;
    constexpr int stride = KIND == 0 ? 2 * D + 1 : KIND == 1 ? 2 * D + 2 : 3 * D + 3;
    int e[4];
    const int n = entries_of(qbn[i], t, e);
    float lo[D][4], hi[D][4], aux[D + 1][4];
    int32_t ref[4], pcs[4];
    int r = 0;
    for (int k = 0; k < 4; ++k) {
        for (int a = 0; a < D; ++a) { lo[a][k] = INFINITY; hi[a][k] = -INFINITY; }
        for (int a = 0; a <= D; ++a) aux[a][k] = 0.f;
        ref[k] = kEmptyRef;
        pcs[k] = -1;
        if (k >= n) continue;
        const int k2 = e[k];
        for (int a = 0; a < D; ++a) {
            lo[a][k] = f_down(f_unord(t.nbox[(int64_t)k2 * 6 + a]));
            hi[a][k] = f_up(f_unord(t.nbox[(int64_t)k2 * 6 + 3 + a]));
        }
        if (t.ncount[k2] > 0) {
            ref[k] = leaf_ref(t.nc[k2], t.ncount[k2]);
        } else {
            const int slot = (int)offs[i] + r++;
            ref[k] = base + slot;
            nqbn[slot] = t.nc[k2];
            nqme[slot] = base + slot;
        }
        if (KIND == 1) aux[0][k] = (float)x.sub_meas[k2];
        if (KIND == 2) {
            for (int a = 0; a < D; ++a) aux[a][k] = (float)x.axis[(int64_t)k2 * 3 + a];
            const double w = d_unord(x.worst[k2]);
            const bool off = x.sub_bnd[k2] || !x.valid[k2] || !(w > 0.0);
            aux[D][k] = off ? -1.f : f_down((float)w);
            pcs[k] = x.sub_piece[k2];
        }
    }
    float4* o = nodes + (int64_t)qme[i] * stride;
    for (int a = 0; a < D; ++a) {
        o[a] = make_float4(lo[a][0], lo[a][1], lo[a][2], lo[a][3]);
        o[D + a] = make_float4(hi[a][0], hi[a][1], hi[a][2], hi[a][3]);
    }
    o[2 * D] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]),
                           __int_as_float(ref[3]));
    if (KIND == 1) o[2 * D + 1] = make_float4(aux[0][0], aux[0][1], aux[0][2], aux[0][3]);
    if (KIND == 2) {
        for (int a = 0; a <= D; ++a) o[2 * D + 1 + a] = make_float4(aux[a][0], aux[a][1], aux[a][2], aux[a][3]);
        o[3 * D + 2] = make_float4(__int_as_float(pcs[0]), __int_as_float(pcs[1]), __int_as_float(pcs[2]),
                                   __int_as_float(pcs[3]));
    }
}

__global__ void gb_c4_root(int32_t* qbn, int32_t* qme)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) { qbn[0] = 0; qme[0] = 0; }
}

// ------------------------------------------------------------ primitive records

// Dirichlet / Neumann records in leaf order, caller indices, Neumann extras
// and the caller -> internal Neumann id table
template <int D, bool NEU>
__global__ __launch_bounds__(kT) void gb_prim_records(int m, const int32_t* perm, const int32_t* list,
                                                      const float* verts, const int32_t* prims, const double* nout,
                                                      const double* meas, float4* out, float4* pextra, int32_t* orig,
                                                      int32_t* neu_id)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    const int q = list[perm[p]];
    float v[3][3];
    for (int k = 0; k < D; ++k) {
        const int32_t vid = prims[(int64_t)q * D + k];
        for (int a = 0; a < D; ++a) v[k][a] = verts[(int64_t)vid * D + a];
    }
    if (D == 2) {
        out[p] = make_float4(v[0][0], v[0][1], v[1][0], v[1][1]);
    } else {
        out[3 * (int64_t)p] = make_float4(v[0][0], v[0][1], v[0][2 % D], v[1][0]);
        out[3 * (int64_t)p + 1] = make_float4(v[1][1], v[1][2 % D], v[D - 1][0], v[D - 1][1]);
        out[3 * (int64_t)p + 2] = make_float4(v[D - 1][2 % D], 0.f, 0.f, 0.f);
    }
    orig[p] = q;
    if (NEU) {
        pextra[p] = make_float4((float)nout[(int64_t)q * 3], (float)nout[(int64_t)q * 3 + 1],
                                (float)nout[(int64_t)q * 3 + 2], (float)meas[q]);
        neu_id[q] = p;
    }
}

// ------------------------------------------------------------ silhouette candidates

// one entry per (Neumann primitive, vertex) in 2D, per (Neumann primitive,
// edge) in 3D; the 3D key sorts by the larger vertex first, then (stably) by
// the smaller one
template <int D>
__global__ __launch_bounds__(kT) void gb_entries(const int32_t* prims, const int32_t* list_neu, int n_neu,
                                                 uint32_t* keys, int32_t* vals)
{
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= D * n_neu) return;
    const int i = e / D, k = e % D;
    const int q = list_neu[i];
    const int32_t a = prims[(int64_t)q * D + k];
    if (D == 2) {
        keys[e] = (uint32_t)a;
    } else {
        const int32_t b = prims[(int64_t)q * D + (k + 1) % D];
        keys[e] = (uint32_t)max(a, b);
    }
    vals[e] = e;
}

template <int D>
__device__ __forceinline__ void entry_edge(const int32_t* prims, const int32_t* list_neu, int e, int32_t& lo,
                                           int32_t& hi)
{
    const int q = list_neu[e / D], k = e % D;
    const int32_t a = prims[(int64_t)q * D + k];
    const int32_t b = D == 2 ? a : prims[(int64_t)q * D + (k + 1) % D];
    lo = min(a, b);
    hi = max(a, b);
}

template <int D>
__global__ __launch_bounds__(kT) void gb_entries_lo(const int32_t* prims, const int32_t* list_neu, int E,
                                                    const int32_t* sorted, uint32_t* keys, int32_t* vals)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= E) return;
    int32_t lo, hi;
    entry_edge<D>(prims, list_neu, sorted[p], lo, hi);
    keys[p] = (uint32_t)lo;
    vals[p] = sorted[p];
}

template <int D>
__global__ __launch_bounds__(kT) void gb_heads(const int32_t* prims, const int32_t* list_neu, int E,
                                               const int32_t* sorted, uint32_t* head)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= E) return;
    int32_t lo, hi, lo0, hi0;
    entry_edge<D>(prims, list_neu, sorted[p], lo, hi);
    if (p == 0) { head[p] = 1; return; }
    entry_edge<D>(prims, list_neu, sorted[p - 1], lo0, hi0);
    head[p] = lo != lo0 || hi != hi0;
}

struct CandBufs {
    int32_t* va;        // [C] vertex (2D) / edge vertices (3D)
    int32_t* vb;
    int32_t* q1;        // [C] caller index of the first / second Neumann neighbour (-1: none)
    int32_t* q2;
    int32_t* bnd;
    int32_t* link;      // [C] 2D: the vertex links its two segments
    int32_t* piece;
    double* n1;         // [C][3]
    double* n2;
};

// a run of equal keys is one candidate: its first two entries are its
// neighbours (a single entry: a boundary feature).  2D: a vertex with exactly
// two segments, one ending and one starting there, strictly convex, normals
// in one quadrant, links them.
template <int D>
__global__ __launch_bounds__(kT) void gb_candidates(const int32_t* prims, const float* verts,
                                                    const int32_t* list_neu, int E, const int32_t* sorted,
                                                    const uint32_t* head, const uint32_t* index, const double* nout,
                                                    CandBufs c, int32_t* jump)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= E || !head[p]) return;
    const int k = (int)index[p];
    int32_t lo, hi;
    entry_edge<D>(prims, list_neu, sorted[p], lo, hi);
    const int q1 = list_neu[sorted[p] / D];
    bool second = false;
    int q2 = -1;
    if (p + 1 < E && !head[p + 1]) { second = true; q2 = list_neu[sorted[p + 1] / D]; }
    const bool exactly_two = second && (p + 2 >= E || head[p + 2]);
    c.va[k] = lo;
    c.vb[k] = hi;
    c.q1[k] = q1;
    c.q2[k] = q2;
    c.bnd[k] = !second;
    for (int a = 0; a < 3; ++a) {
        c.n1[(int64_t)k * 3 + a] = -nout[(int64_t)q1 * 3 + a];
        c.n2[(int64_t)k * 3 + a] = second ? -nout[(int64_t)q2 * 3 + a] : 0.0;
    }
    int link = 0;
    if (D == 2 && exactly_two) {
        const int v = lo, s1 = q1, s2 = q2;
        const bool end1 = prims[(int64_t)s1 * 2 + 1] == v, end2 = prims[(int64_t)s2 * 2 + 1] == v;
        if (end1 != end2) {
            const int p1 = end1 ? prims[(int64_t)s1 * 2] : prims[(int64_t)s1 * 2 + 1];
            const int p2 = end2 ? prims[(int64_t)s2 * 2] : prims[(int64_t)s2 * 2 + 1];
            double e1[2], e2[2];
            for (int i = 0; i < 2; ++i) {
                e1[i] = (double)verts[(int64_t)p1 * 2 + i] - (double)verts[(int64_t)v * 2 + i];
                e2[i] = (double)verts[(int64_t)p2 * 2 + i] - (double)verts[(int64_t)v * 2 + i];
            }
            const double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1]);
            const double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1]);
            const double* m1 = nout + (int64_t)s1 * 3;
            const double* m2 = nout + (int64_t)s2 * 3;
            const double c1 = -(e2[0] * m1[0] + e2[1] * m1[1]) / l2;
            const double c2 = -(e1[0] * m2[0] + e1[1] * m2[1]) / l1;
            const int quad1 = m1[0] >= 0 ? (m1[1] >= 0 ? 0 : 3) : (m1[1] >= 0 ? 1 : 2);
            const int quad2 = m2[0] >= 0 ? (m2[1] >= 0 ? 0 : 3) : (m2[1] >= 0 ? 1 : 2);
            if (c1 > 1e-6 && c2 > 1e-6 && quad1 == quad2) {
                link = 1;
                if (end1) jump[s1] = s2;
                else jump[s2] = s1;
            }
        }
    }
    c.link[k] = link;
}

__global__ __launch_bounds__(kT) void gb_jump_init(const uint8_t* bc, int P, int32_t* jump)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q < P) jump[q] = bc[q] ? q : -1;
}

__global__ __launch_bounds__(kT) void gb_jump(const int32_t* in, int P, int32_t* out)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    if (q < P) out[q] = in[q] >= 0 ? in[in[q]] : -1;
}

template <int D>
__global__ __launch_bounds__(kT) void gb_cand_items(int C, const float* verts, const int32_t* seg_piece, CandBufs c,
                                                    int ms, float* blo, float* bhi, double* cen)
{
    const int k = blockIdx.x * kT + threadIdx.x;
    if (k >= C) return;
    const int va = c.va[k], vb = D == 2 ? c.va[k] : c.vb[k];
    for (int a = 0; a < D; ++a) {
        const float x = verts[(int64_t)va * D + a], y = verts[(int64_t)vb * D + a];
        const float lo = fminf(x, y), hi = fmaxf(x, y);
        blo[(int64_t)a * ms + k] = lo;
        bhi[(int64_t)a * ms + k] = hi;
        cen[(int64_t)a * ms + k] = 0.5 * ((double)lo + (double)hi);
    }
    c.piece[k] = D == 2 && c.link[k] && seg_piece ? seg_piece[c.q1[k]] : -1;
}

template <int D>
__global__ __launch_bounds__(kT) void gb_sil_records(int m, const int32_t* perm, const float* verts, CandBufs c,
                                                     const int32_t* neu_id, float4* out)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p >= m) return;
    const int k = perm[p];
    const float f1 = __int_as_float(neu_id[c.q1[k]]);
    const float f2 = __int_as_float(c.q2[k] >= 0 ? neu_id[c.q2[k]] : -1);
    const double* n1 = c.n1 + (int64_t)k * 3;
    const double* n2 = c.n2 + (int64_t)k * 3;
    const int va = c.va[k], vb = c.vb[k];
    if (D == 2) {
        out[2 * (int64_t)p] = make_float4(verts[(int64_t)va * 2], verts[(int64_t)va * 2 + 1], (float)n1[0], (float)n1[1]);
        out[2 * (int64_t)p + 1] = make_float4((float)n2[0], (float)n2[1], f1, f2);
    } else {
        const float* a = verts + (int64_t)va * D;
        const float* b = verts + (int64_t)vb * D;
        out[4 * (int64_t)p] = make_float4(a[0], a[1], a[2 % D], b[0]);
        out[4 * (int64_t)p + 1] = make_float4(b[1], b[2 % D], (float)n1[0], (float)n1[1]);
        out[4 * (int64_t)p + 2] = make_float4((float)n1[2], (float)n2[0], (float)n2[1], (float)n2[2]);
        out[4 * (int64_t)p + 3] = make_float4(f1, f2, 0.f, 0.f);
    }
}

// convex piece of every Neumann primitive by internal id
__global__ __launch_bounds__(kT) void gb_piece_table(int n_neu, const int32_t* orig_neu, const int32_t* seg_piece,
                                                     int32_t* out)
{
    const int p = blockIdx.x * kT + threadIdx.x;
    if (p < n_neu) out[p] = seg_piece ? seg_piece[orig_neu[p]] : -1;
}

}  // namespace
}  // namespace wost

// ================================================================== host side

namespace wost {
namespace {

struct Ws {
    // inputs, per primitive
    int32_t* list;      // [P] caller indices: Dirichlet then Neumann, each ascending
    double* nout;       // [P][3]
    double* meas;       // [P]
    int32_t* jump;      // [P] 2D piece pointers
    int32_t* jump2;
    double* imeas;      // [P] Neumann item measures
    unsigned long long* err;
    uint32_t* counters; // [16]
    uint32_t* vb;       // [6] ordered vertex bounds
    // items
    float *blo, *bhi;   // [3][ms]
    double* cen;        // [3][ms]
    uint32_t* rank;     // [3][ms]
    int32_t* perm;      // [ms] position -> item
    uint32_t *keys_a, *keys_b, *key2;
    int32_t *vals_a, *vals_b, *pslot;
    uint32_t* hist;
    int32_t *rb[2], *re[2], *rnode[2], *rax;
    uint32_t* oc;
    uint64_t* cbox;
    TreeBufs t;
    int32_t* lvl;       // [nn] inner nodes level by level
    double *sub_meas, *node_meas;
    SilAgg g;
    int32_t *qbn[2], *qme[2];
    uint32_t* qcnt;
    CandBufs c;
    uint32_t *head, *index;
    // outputs (the image's arrays, staged)
    float4 *dir_nodes, *dir_prims, *neu_nodes, *neu_prims, *neu_extra, *sil_nodes, *sil_prims;
    int32_t *dir_orig, *neu_orig, *sil_piece, *neu_id;
    int64_t ms;         // item capacity
    int64_t nn_cap;     // inner-node capacity
};

inline int64_t a256(int64_t v) { return (v + 255) & ~int64_t(255); }

int64_t ws_layout(int d, int64_t P, int L, uint8_t* base, Ws* w)
{
    const int64_t Pc = std::max<int64_t>(P, 1);
    const int64_t C = d * Pc;                 // silhouette entries / candidates bound
    const int64_t ms = C;                     // items bound (>= P)
    const int64_t nn = std::max<int64_t>(inner_count(ms, L), 1);
    const int64_t nn_p = std::max<int64_t>(inner_count(Pc, L), 1);
    const int pf = d == 2 ? 1 : 3, sf = d == 2 ? 2 : 4;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { const int64_t o = off; off += a256(std::max<int64_t>(bytes, 1)); return base ? base + o : nullptr; };
    Ws t{};
    t.ms = ms;
    t.nn_cap = nn;
    t.list = (int32_t*)take(Pc * 4);
    t.nout = (double*)take(Pc * 24);
    t.meas = (double*)take(Pc * 8);
    t.jump = (int32_t*)take(Pc * 4);
    t.jump2 = (int32_t*)take(Pc * 4);
    t.imeas = (double*)take(Pc * 8);
    t.err = (unsigned long long*)take(8);
    t.counters = (uint32_t*)take(64);
    t.vb = (uint32_t*)take(24);
    t.blo = (float*)take(3 * ms * 4);
    t.bhi = (float*)take(3 * ms * 4);
    t.cen = (double*)take(3 * ms * 8);
    t.rank = (uint32_t*)take(3 * ms * 4);
    t.perm = (int32_t*)take(ms * 4);
    t.keys_a = (uint32_t*)take(ms * 4);
    t.keys_b = (uint32_t*)take(ms * 4);
    t.key2 = (uint32_t*)take(ms * 4);
    t.vals_a = (int32_t*)take(ms * 4);
    t.vals_b = (int32_t*)take(ms * 4);
    t.pslot = (int32_t*)take(ms * 4);
    t.hist = (uint32_t*)take(rs_hist_words(ms) * 4);
    for (int k = 0; k < 2; ++k) {
        t.rb[k] = (int32_t*)take(ms * 4);
        t.re[k] = (int32_t*)take(ms * 4);
        t.rnode[k] = (int32_t*)take(ms * 4);
    }
    t.rax = (int32_t*)take(ms * 4);
    t.oc = (uint32_t*)take(ms * 4);
    t.cbox = (uint64_t*)take(ms * 6 * 8);
    t.t.nc = (int32_t*)take(2 * nn * 4);
    t.t.ncount = (int32_t*)take(2 * nn * 4);
    t.t.parent = (int32_t*)take(nn * 4);
    t.t.nbox = (uint32_t*)take(2 * nn * 6 * 4);
    t.t.leaves = (int32_t*)take(3 * ms * 4);
    t.t.pleaf = (int32_t*)take(ms * 4);
    t.t.counters = t.counters + 8;
    t.lvl = (int32_t*)take(nn * 4);
    t.sub_meas = (double*)take(2 * nn * 8);
    t.node_meas = (double*)take(nn * 8);
    t.g.sub_sum = (double*)take(2 * nn * 24);
    t.g.node_sum = (double*)take(nn * 24);
    t.g.sub_cnt = (int32_t*)take(2 * nn * 4);
    t.g.node_cnt = (int32_t*)take(nn * 4);
    t.g.sub_bnd = (int32_t*)take(2 * nn * 4);
    t.g.node_bnd = (int32_t*)take(nn * 4);
    t.g.sub_piece = (int32_t*)take(2 * nn * 4);
    t.g.node_piece = (int32_t*)take(nn * 4);
    t.g.axis = (double*)take(2 * nn * 24);
    t.g.valid = (int32_t*)take(2 * nn * 4);
    t.g.worst = (uint64_t*)take(2 * nn * 8);
    for (int k = 0; k < 2; ++k) {
        t.qbn[k] = (int32_t*)take(nn * 4);
        t.qme[k] = (int32_t*)take(nn * 4);
    }
    t.qcnt = (uint32_t*)take(nn * 4);
    t.c.va = (int32_t*)take(C * 4);
    t.c.vb = (int32_t*)take(C * 4);
    t.c.q1 = (int32_t*)take(C * 4);
    t.c.q2 = (int32_t*)take(C * 4);
    t.c.bnd = (int32_t*)take(C * 4);
    t.c.link = (int32_t*)take(C * 4);
    t.c.piece = (int32_t*)take(C * 4);
    t.c.n1 = (double*)take(C * 24);
    t.c.n2 = (double*)take(C * 24);
    t.head = (uint32_t*)take(C * 4);
    t.index = (uint32_t*)take(C * 4);
    t.dir_nodes = (float4*)take(nn_p * (2 * d + 1) * 16);
    t.dir_prims = (float4*)take(Pc * pf * 16);
    t.dir_orig = (int32_t*)take(Pc * 4);
    t.neu_nodes = (float4*)take(nn_p * (2 * d + 2) * 16);
    t.neu_prims = (float4*)take(Pc * pf * 16);
    t.neu_extra = (float4*)take(Pc * 16);
    t.neu_orig = (int32_t*)take(Pc * 4);
    t.sil_nodes = (float4*)take(nn * (3 * d + 3) * 16);
    t.sil_prims = (float4*)take(C * sf * 16);
    t.sil_piece = (int32_t*)take(Pc * 4);
    t.neu_id = (int32_t*)take(Pc * 4);
    if (w) *w = t;
    return off;
}

int sync_read(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("wost_build_bvh_device: %s", hipGetErrorString(hipGetLastError()));
        return WOST_EHIP;
    }
    return WOST_OK;
}

struct Tree {
    int nn = 0;             // binary inner nodes
    int max_depth = 0;      // deepest leaf (the host's split depth)
    std::vector<int> lvl_off;
};

// median-split hierarchy over the m items in w.blo/bhi/cen (capacity w.ms)
template <int D>
int build_tree(const Ws& w, int m, int L, hipStream_t s, Tree& out)
{
    out = Tree{};
    if (m == 0) return WOST_OK;
    const int ms = (int)w.ms;
    out.nn = m <= L ? 1 : (int)inner_count(m, L);
    for (int a = 0; a < D; ++a) {
        hipLaunchKernelGGL(gb_rank_lo, dim3(blocks(m)), dim3(kT), 0, s, w.cen + (int64_t)a * ms, m, w.keys_a, w.vals_a);
        if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, m, 32, w.hist, s) != WOST_OK) return WOST_EHIP;
        hipLaunchKernelGGL(gb_rank_hi, dim3(blocks(m)), dim3(kT), 0, s, w.cen + (int64_t)a * ms, w.vals_b, m, w.keys_a,
                           w.vals_a);
        if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, m, 32, w.hist, s) != WOST_OK) return WOST_EHIP;
        hipLaunchKernelGGL(gb_rank_store, dim3(blocks(m)), dim3(kT), 0, s, w.vals_b, m, w.rank + (int64_t)a * ms);
    }
    hipLaunchKernelGGL(gb_fill_u32, dim3(1), dim3(kT), 0, s, w.t.counters, (int64_t)4, 0u);
    hipLaunchKernelGGL(gb_box_init, dim3(blocks(2 * (int64_t)out.nn)), dim3(kT), 0, s, w.t.nbox, 2 * (int64_t)out.nn);
    hipLaunchKernelGGL(gb_iota, dim3(blocks(m)), dim3(kT), 0, s, w.perm, m);
    hipLaunchKernelGGL(gb_fill_i32, dim3(1), dim3(kT), 0, s, w.lvl, (int64_t)1, 0);
    hipLaunchKernelGGL(gb_fill_i32, dim3(1), dim3(kT), 0, s, w.t.parent, (int64_t)1, -1);
    out.lvl_off = {0, 1};
    if (m <= L) {
        hipLaunchKernelGGL(gb_root_leaf, dim3(1), dim3(64), 0, s, m, w.t);
        hipLaunchKernelGGL(gb_root_box<D>, dim3(blocks(m)), dim3(kT), 0, s, m, w.blo, w.bhi, ms, w.t.nbox);
    } else {
        hipLaunchKernelGGL(gb_fill_i32, dim3(1), dim3(kT), 0, s, w.rb[0], (int64_t)1, 0);
        hipLaunchKernelGGL(gb_fill_i32, dim3(1), dim3(kT), 0, s, w.re[0], (int64_t)1, m);
        hipLaunchKernelGGL(gb_fill_i32, dim3(1), dim3(kT), 0, s, w.rnode[0], (int64_t)1, 0);
        int R = 1, cur = 0;
        for (int depth = 0; R > 0; ++depth) {
            if (depth > 62) { set_error("wost_build_bvh_device: internal error: split depth"); return WOST_EINVAL; }
            const int32_t *rb = w.rb[cur], *re = w.re[cur], *rn = w.rnode[cur];
            hipLaunchKernelGGL(gb_level_pos, dim3(blocks(m)), dim3(kT), 0, s, m, rb, re, R, w.perm, w.pslot, w.key2);
            hipLaunchKernelGGL(gb_cbox_init<D>, dim3(blocks(R)), dim3(kT), 0, s, w.cbox, R);
            hipLaunchKernelGGL(gb_cbox<D>, dim3(blocks(m)), dim3(kT), 0, s, m, w.pslot, w.perm, w.cen, ms, w.cbox);
            hipLaunchKernelGGL(gb_axis<D>, dim3(blocks(R)), dim3(kT), 0, s, R, w.cbox, w.rax);
            hipLaunchKernelGGL(gb_level_keys, dim3(blocks(m)), dim3(kT), 0, s, m, w.pslot, w.perm, w.rax, w.rank, ms,
                               w.keys_a, w.vals_a);
            if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, m, bits_for(m), w.hist, s) != WOST_OK)
                return WOST_EHIP;
            hipLaunchKernelGGL(gb_level_keys2, dim3(blocks(m)), dim3(kT), 0, s, m, w.vals_b, w.key2, w.keys_a,
                               w.vals_a);
            if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, m, bits_for(2 * (int64_t)R + 2), w.hist, s) !=
                WOST_OK)
                return WOST_EHIP;
            hipLaunchKernelGGL(gb_copy_i32, dim3(blocks(m)), dim3(kT), 0, s, w.vals_b, w.perm, m);
            hipLaunchKernelGGL(gb_children, dim3(blocks(R)), dim3(kT), 0, s, R, rb, re, rn, L, depth, w.t, w.oc);
            hipLaunchKernelGGL(gb_child_boxes<D>, dim3(blocks(m)), dim3(kT), 0, s, m, w.pslot, rb, re, rn, w.perm,
                               w.blo, w.bhi, ms, w.t.nbox);
            hipLaunchKernelGGL(rs_scan, dim3(1), dim3(1024), 0, s, w.oc, R, w.t.counters + 2);
            uint32_t rn_next = 0;
            if (sync_read(&rn_next, w.t.counters + 2, 4, s) != WOST_OK) return WOST_EHIP;
            const int nxt = cur ^ 1;
            hipLaunchKernelGGL(gb_next_ranges, dim3(blocks(R)), dim3(kT), 0, s, R, rb, re, rn, L, w.oc, w.rb[nxt],
                               w.re[nxt], w.rnode[nxt], w.lvl + out.lvl_off.back());
            if (rn_next > 0) out.lvl_off.push_back(out.lvl_off.back() + (int)rn_next);
            cur = nxt;
            R = (int)rn_next;
        }
        if (out.lvl_off.back() != out.nn) {
            set_error("wost_build_bvh_device: internal error: %d inner nodes, expected %d", out.lvl_off.back(), out.nn);
            return WOST_EINVAL;
        }
    }
    uint32_t cnt[2] = {0, 0};
    if (sync_read(cnt, w.t.counters, 8, s) != WOST_OK) return WOST_EHIP;
    out.max_depth = (int)cnt[1];
    hipLaunchKernelGGL(gb_leaf_sort, dim3(blocks(cnt[0])), dim3(kT), 0, s, (int)cnt[0], w.t.leaves, w.perm);
    return hipGetLastError() == hipSuccess ? WOST_OK : WOST_EHIP;
}

// four-wide collapse breadth first; returns the node count and level count
template <int D, int KIND>
int collapse(const Ws& w, const Tree& tr, const C4Aux& x, float4* nodes, hipStream_t s, int& n4, int& levels4)
{
    n4 = 0;
    levels4 = 0;
    if (tr.nn == 0) return WOST_OK;
    hipLaunchKernelGGL(gb_c4_root, dim3(1), dim3(64), 0, s, w.qbn[0], w.qme[0]);
    int Q = 1, base = 1, cur = 0;
    while (Q > 0) {
        if (levels4 >= 64) { set_error("wost_build_bvh_device: internal error: four-wide depth"); return WOST_EINVAL; }
        hipLaunchKernelGGL(gb_c4_count, dim3(blocks(Q)), dim3(kT), 0, s, Q, w.qbn[cur], w.t, w.qcnt);
        hipLaunchKernelGGL(rs_scan, dim3(1), dim3(1024), 0, s, w.qcnt, Q, w.t.counters + 2);
        uint32_t total = 0;
        if (sync_read(&total, w.t.counters + 2, 4, s) != WOST_OK) return WOST_EHIP;
        hipLaunchKernelGGL((gb_c4_write<D, KIND>), dim3(blocks(Q)), dim3(kT), 0, s, Q, w.qbn[cur], w.qme[cur], w.qcnt,
                           base, w.t, x, nodes, w.qbn[cur ^ 1], w.qme[cur ^ 1]);
        base += (int)total;
        Q = (int)total;
        cur ^= 1;
        ++levels4;
    }
    n4 = base;
    return hipGetLastError() == hipSuccess ? WOST_OK : WOST_EHIP;
}

template <int D>
int build_all(const float* verts, int64_t V, const int32_t* prims, int P, const uint8_t* bc, int L, const Ws& w,
              hipStream_t s, wost_geom* g)
{
    const int ms = (int)w.ms;
    // ---- validation, normals, measures, vertex bounds
    if (hipMemsetAsync(w.err, 0xFF, 8, s) != hipSuccess) return WOST_EHIP;
    hipLaunchKernelGGL(gb_fill_u32, dim3(1), dim3(kT), 0, s, w.counters, (int64_t)16, 0u);
    hipLaunchKernelGGL(gb_fill_u32, dim3(1), dim3(kT), 0, s, w.vb, (int64_t)3, ~0u);
    hipLaunchKernelGGL(gb_fill_u32, dim3(1), dim3(kT), 0, s, w.vb + 3, (int64_t)3, 0u);
    hipLaunchKernelGGL(gb_verts<D>, dim3(blocks(V)), dim3(kT), 0, s, verts, V, w.vb, w.err);
    hipLaunchKernelGGL(gb_prims<D>, dim3(blocks(P)), dim3(kT), 0, s, verts, V, prims, P, bc, w.nout, w.meas, w.counters,
                       w.err);
    unsigned long long err = 0;
    uint32_t vb[6], n_neu_u = 0;
    if (sync_read(&err, w.err, 8, s) != WOST_OK || sync_read(vb, w.vb, 24, s) != WOST_OK ||
        sync_read(&n_neu_u, w.counters, 4, s) != WOST_OK)
        return WOST_EHIP;
    if (err != ~0ull) {
        const int stage = (int)(err >> 60), kind = (int)(err & 15);
        const long long idx = (long long)((err >> 4) & ((1ull << 56) - 1));
        if (stage == 0) set_error("wost_build_bvh_device: non-finite vertex %lld", idx);
        else if (kind == 1) set_error("wost_build_bvh_device: bc[%lld] must be 0 or 1", idx);
        else if (kind == 2) set_error("wost_build_bvh_device: prim %lld references a vertex out of range", idx);
        else set_error("wost_build_bvh_device: degenerate %s %lld", D == 2 ? "segment" : "triangle", idx);
        return WOST_EINVAL;
    }
    const int n_neu = (int)n_neu_u, n_dir = P - n_neu;
    for (int a = 0; a < 3; ++a) {
        auto unord = [](uint32_t u) {
            uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
            float f;
            memcpy(&f, &b, 4);
            return f;
        };
        g->lo[a] = a < D ? (double)unord(vb[a]) : 0.0;
        g->hi[a] = a < D ? (double)unord(vb[3 + a]) : 0.0;
    }
    double diag2 = 0;
    for (int a = 0; a < D; ++a) diag2 += (g->hi[a] - g->lo[a]) * (g->hi[a] - g->lo[a]);
    g->diag = std::sqrt(diag2);
    // ---- classes: Dirichlet then Neumann, caller order within each
    hipLaunchKernelGGL(gb_class_keys, dim3(blocks(P)), dim3(kT), 0, s, bc, P, w.keys_a, w.vals_a);
    if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, P, 1, w.hist, s) != WOST_OK) return WOST_EHIP;
    hipLaunchKernelGGL(gb_copy_i32, dim3(blocks(P)), dim3(kT), 0, s, w.vals_b, w.list, P);
    const int32_t* list_neu = w.list + n_dir;
    hipLaunchKernelGGL(gb_fill_i32, dim3(blocks(P)), dim3(kT), 0, s, w.neu_id, (int64_t)P, -1);

    int sec_nodes[3], sec_levels[3], max_depth = 0;
    // ---- Dirichlet hierarchy
    {
        hipLaunchKernelGGL(gb_items_prims<D>, dim3(blocks(n_dir)), dim3(kT), 0, s, verts, prims, w.list, n_dir, ms,
                           w.blo, w.bhi, w.cen);
        Tree tr;
        int rc = build_tree<D>(w, n_dir, L, s, tr);
        if (rc != WOST_OK) return rc;
        max_depth = std::max(max_depth, tr.max_depth);
        rc = collapse<D, 0>(w, tr, C4Aux{}, w.dir_nodes, s, sec_nodes[0], sec_levels[0]);
        if (rc != WOST_OK) return rc;
        hipLaunchKernelGGL((gb_prim_records<D, false>), dim3(blocks(n_dir)), dim3(kT), 0, s, n_dir, w.perm, w.list,
                           verts, prims, w.nout, w.meas, w.dir_prims, (float4*)nullptr, w.dir_orig, (int32_t*)nullptr);
    }
    // ---- Neumann hierarchy with subtree measures
    {
        hipLaunchKernelGGL(gb_items_prims<D>, dim3(blocks(n_neu)), dim3(kT), 0, s, verts, prims, list_neu, n_neu, ms,
                           w.blo, w.bhi, w.cen);
        Tree tr;
        int rc = build_tree<D>(w, n_neu, L, s, tr);
        if (rc != WOST_OK) return rc;
        max_depth = std::max(max_depth, tr.max_depth);
        hipLaunchKernelGGL(gb_gather_meas, dim3(blocks(n_neu)), dim3(kT), 0, s, list_neu, n_neu, w.meas, w.imeas);
        for (int l = (int)tr.lvl_off.size() - 2; l >= 0; --l) {
            const int cnt = tr.lvl_off[l + 1] - tr.lvl_off[l];
            hipLaunchKernelGGL(gb_agg_neu, dim3(blocks(cnt)), dim3(kT), 0, s, w.lvl + tr.lvl_off[l], cnt, w.t, w.perm,
                               w.imeas, w.sub_meas, w.node_meas);
        }
        C4Aux x{};
        x.sub_meas = w.sub_meas;
        rc = collapse<D, 1>(w, tr, x, w.neu_nodes, s, sec_nodes[1], sec_levels[1]);
        if (rc != WOST_OK) return rc;
        hipLaunchKernelGGL((gb_prim_records<D, true>), dim3(blocks(n_neu)), dim3(kT), 0, s, n_neu, w.perm, list_neu,
                           verts, prims, w.nout, w.meas, w.neu_prims, w.neu_extra, w.neu_orig, w.neu_id);
    }
    // ---- silhouette candidates
    int n_sil = 0;
    const int E = D * n_neu;
    if (D == 2) {
        hipLaunchKernelGGL(gb_jump_init, dim3(blocks(P)), dim3(kT), 0, s, bc, P, w.jump);
    }
    if (E > 0) {
        hipLaunchKernelGGL(gb_entries<D>, dim3(blocks(E)), dim3(kT), 0, s, prims, list_neu, n_neu, w.keys_a, w.vals_a);
        if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, E, bits_for(V), w.hist, s) != WOST_OK) return WOST_EHIP;
        if (D == 3) {
            hipLaunchKernelGGL(gb_entries_lo<D>, dim3(blocks(E)), dim3(kT), 0, s, prims, list_neu, E, w.vals_b, w.keys_a,
                               w.vals_a);
            if (rs_sort_pairs(w.keys_a, w.vals_a, w.keys_b, w.vals_b, E, bits_for(V), w.hist, s) != WOST_OK)
                return WOST_EHIP;
        }
        hipLaunchKernelGGL(gb_heads<D>, dim3(blocks(E)), dim3(kT), 0, s, prims, list_neu, E, w.vals_b, w.head);
        hipLaunchKernelGGL(gb_copy_i32, dim3(blocks(E)), dim3(kT), 0, s, (const int32_t*)w.head, (int32_t*)w.index, E);
        hipLaunchKernelGGL(rs_scan, dim3(1), dim3(1024), 0, s, w.index, E, w.counters + 4);
        uint32_t c = 0;
        if (sync_read(&c, w.counters + 4, 4, s) != WOST_OK) return WOST_EHIP;
        n_sil = (int)c;
        hipLaunchKernelGGL(gb_candidates<D>, dim3(blocks(E)), dim3(kT), 0, s, prims, verts, list_neu, E, w.vals_b,
                           w.head, w.index, w.nout, w.c, w.jump);
    }
    const int32_t* seg_piece = nullptr;
    if (D == 2) {
        int rounds = 1;
        while ((int64_t(1) << rounds) < (int64_t)n_neu + 1) ++rounds;
        int32_t* a = w.jump;
        int32_t* b = w.jump2;
        for (int r = 0; r < rounds; ++r) {
            hipLaunchKernelGGL(gb_jump, dim3(blocks(P)), dim3(kT), 0, s, a, P, b);
            std::swap(a, b);
        }
        seg_piece = a;
    }
    // ---- silhouette hierarchy with normal cones and convex pieces
    {
        hipLaunchKernelGGL(gb_cand_items<D>, dim3(blocks(n_sil)), dim3(kT), 0, s, n_sil, verts, seg_piece, w.c, ms,
                           w.blo, w.bhi, w.cen);
        Tree tr;
        int rc = build_tree<D>(w, n_sil, L, s, tr);
        if (rc != WOST_OK) return rc;
        max_depth = std::max(max_depth, tr.max_depth);
        SilItems it{w.c.n1, w.c.n2, w.c.bnd, w.c.piece};
        for (int l = (int)tr.lvl_off.size() - 2; l >= 0 && tr.nn > 0; --l) {
            const int cnt = tr.lvl_off[l + 1] - tr.lvl_off[l];
            hipLaunchKernelGGL(gb_agg_sil, dim3(blocks(cnt)), dim3(kT), 0, s, w.lvl + tr.lvl_off[l], cnt, w.t, w.perm,
                               it, w.g);
        }
        if (tr.nn > 0) {
            hipLaunchKernelGGL(gb_axes, dim3(blocks(2 * tr.nn)), dim3(kT), 0, s, 2 * tr.nn, w.g);
            hipLaunchKernelGGL(gb_worst, dim3(blocks(n_sil)), dim3(kT), 0, s, n_sil, w.perm, w.t, it, w.g);
        }
        C4Aux x{};
        x.axis = w.g.axis;
        x.valid = w.g.valid;
        x.worst = w.g.worst;
        x.sub_bnd = w.g.sub_bnd;
        x.sub_piece = w.g.sub_piece;
        rc = collapse<D, 2>(w, tr, x, w.sil_nodes, s, sec_nodes[2], sec_levels[2]);
        if (rc != WOST_OK) return rc;
        hipLaunchKernelGGL(gb_sil_records<D>, dim3(blocks(n_sil)), dim3(kT), 0, s, n_sil, w.perm, verts, w.c, w.neu_id,
                           w.sil_prims);
        hipLaunchKernelGGL(gb_fill_i32, dim3(1), dim3(kT), 0, s, w.sil_piece, (int64_t)1, -1);
        hipLaunchKernelGGL(gb_piece_table, dim3(blocks(n_neu)), dim3(kT), 0, s, n_neu, w.neu_orig, seg_piece,
                           w.sil_piece);
    }
    // ---- limits the traversals rely on
    const int counts[3] = {n_dir, n_neu, n_sil};
    int stack = 0;
    for (int k = 0; k < 3; ++k) {
        const int need = 3 * std::max(sec_levels[k] - 1, 0) + 1;
        stack = std::max(stack, need);
        if (need > kMaxStack || (int64_t)counts[k] > kMaxLeafFirst) {
            set_error("wost_build_bvh_device: hierarchy %d too deep or too large (stack %d > %d or %d primitives)", k,
                      need, kMaxStack, counts[k]);
            return WOST_EUNSUPPORTED;
        }
    }
    // ---- the image layout of the host builder
    g->dim = D;
    g->n_dir = n_dir;
    g->n_neu = n_neu;
    g->n_sil = n_sil;
    g->max_depth = max_depth;
    g->stack_entries = stack;
    g->n_caller = P;
    int64_t end = 0;
    auto place = [&](const void* src, int64_t bytes) {
        const int64_t off = a256(end);
        end = off + bytes;
        if (bytes > 0) g->staged.push_back({src, off, bytes});
        return off;
    };
    const int pf = D == 2 ? 1 : 3, sf = D == 2 ? 2 : 4;
    const int strides[3] = {2 * D + 1, 2 * D + 2, 3 * D + 3};
    const float4* nodes[3] = {w.dir_nodes, w.neu_nodes, w.sil_nodes};
    const float4* recs[3] = {w.dir_prims, w.neu_prims, w.sil_prims};
    for (int k = 0; k < 3; ++k) {
        auto& sc = g->sec[k];
        sc.nodes = place(nodes[k], (int64_t)sec_nodes[k] * strides[k] * 16);
        sc.prims = place(recs[k], (int64_t)counts[k] * (k == 2 ? sf : pf) * 16);
        sc.pextra = k == 1 ? place(w.neu_extra, (int64_t)n_neu * 16) : -1;
        sc.orig = k < 2 ? place(k == 0 ? w.dir_orig : w.neu_orig, (int64_t)counts[k] * 4) : -1;
        sc.piece = k == 2 ? place(w.sil_piece, std::max<int64_t>(n_neu, 1) * 4) : -1;
        sc.n_nodes = sec_nodes[k];
        sc.n_prims = counts[k];
    }
    g->off_neu_id = place(w.neu_id, (int64_t)P * 4);
    g->bytes = a256(end);
    // caller indices of the internal primitive ids, for wost_geom_prim_index
    g->orig_host = (int32_t*)malloc(sizeof(int32_t) * ((size_t)P + 1));
    if (!g->orig_host) { set_error("wost_build_bvh_device: out of host memory"); return WOST_EINVAL; }
    if ((n_dir > 0 && sync_read(g->orig_host, w.dir_orig, 4 * (size_t)n_dir, s) != WOST_OK) ||
        (n_neu > 0 && sync_read(g->orig_host + n_dir, w.neu_orig, 4 * (size_t)n_neu, s) != WOST_OK))
        return WOST_EHIP;
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_error("wost_build_bvh_device: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

}  // namespace
}  // namespace wost

using namespace wost;

extern "C" int wost_build_bvh_device_workspace(int32_t dim, int64_t n_verts, int64_t n_prims,
                                               const wost_build_opts* opts, int64_t* ws_bytes)
{
    if (!ws_bytes) { set_error("wost_build_bvh_device_workspace: ws_bytes is NULL"); return WOST_EINVAL; }
    if ((dim != 2 && dim != 3) || n_verts <= 0 || n_prims <= 0) {
        set_error("wost_build_bvh_device_workspace: dim 2 or 3 and a non-empty geometry");
        return WOST_EINVAL;
    }
    if (n_prims > kMaxLeafFirst || n_verts >= (1ll << 31)) {
        set_error("wost_build_bvh_device_workspace: at most %lld primitives", (long long)kMaxLeafFirst);
        return WOST_EUNSUPPORTED;
    }
    const int L = opts ? opts->leaf_size : 4;
    if (L < 1 || L > kLeafMax) { set_error("wost_build_bvh_device_workspace: leaf_size in [1, 64]"); return WOST_EINVAL; }
    *ws_bytes = ws_layout(dim, n_prims, L, nullptr, nullptr);
    return WOST_OK;
}

extern "C" int wost_build_bvh_device(int32_t dim, const float* verts, int64_t n_verts, const int32_t* prims,
                                     int64_t n_prims, const uint8_t* bc, const wost_build_opts* opts, void* workspace,
                                     int64_t ws_bytes, void* stream, wost_geom** out)
{
    if (!out) { set_error("wost_build_bvh_device: out is NULL"); return WOST_EINVAL; }
    *out = nullptr;
    int64_t need = 0;
    const int rc0 = wost_build_bvh_device_workspace(dim, n_verts, n_prims, opts, &need);
    if (rc0 != WOST_OK) return rc0;
    if (!verts || !prims || !bc || !workspace) { set_error("wost_build_bvh_device: NULL argument"); return WOST_EINVAL; }
    if (opts && opts->brute_force) {
        set_error("wost_build_bvh_device: brute_force is a host-build option");
        return WOST_EUNSUPPORTED;
    }
    if (ws_bytes < need) {
        set_error("wost_build_bvh_device: workspace %lld < %lld bytes", (long long)ws_bytes, (long long)need);
        return WOST_ESIZE;
    }
    if ((uintptr_t)workspace & 255) { set_error("wost_build_bvh_device: workspace must be 256-byte aligned"); return WOST_EINVAL; }
    const int L = opts ? opts->leaf_size : 4;
    Ws w;
    ws_layout(dim, n_prims, L, (uint8_t*)workspace, &w);
    wost_geom* g = new wost_geom();
    hipStream_t s = (hipStream_t)stream;
    const int rc = dim == 2 ? build_all<2>(verts, n_verts, prims, (int)n_prims, bc, L, w, s, g)
                            : build_all<3>(verts, n_verts, prims, (int)n_prims, bc, L, w, s, g);
    if (rc != WOST_OK) {
        (void)hipStreamSynchronize(s);
        wost_geom_free(g);
        return rc;
    }
    *out = g;
    return WOST_OK;
}
