// Linear BVH built on the GPU (Karras, "Maximizing parallelism in the
// construction of BVHs, octrees, and k-d trees", HPG 2012; the paper's query
// library uses such a hierarchy, Sec. 5.3) for closest-point queries, written
// in the four-wide node layout the walk traversals read.
//
// Build: primitive bounds and centroids -> scene bounds (two-pass reduction)
// -> Morton codes of the centroids -> radix sort of (code, primitive) (own
// stable LSD sort, 8 bits per pass) ->
// binary radix tree, one thread per internal node (equal codes are ordered by
// index) -> node boxes bottom-up, the second child to arrive at a node
// computing its box -> collapse to four-wide nodes level by level: a node
// takes its binary node's two children and keeps splitting the child with the
// most primitives until it has four, and a child with at most leaf_size
// primitives becomes a leaf over its contiguous range of sorted primitives.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <climits>
#include <cstring>

#include "geom_device.h"
#include "radix_sort.h"

namespace wost {
namespace {

constexpr int kBoundsBlocks = 1024;
constexpr int kMaxLbvhLevels = 64;

template <int D> constexpr int prim_f4() { return D == 2 ? 1 : 3; }

template <int D>
__device__ __forceinline__ void prim_box(const float4* prims, int i, float* lo, float* hi)
{
    float v[3][3];
    int nv;
    if (D == 2) {
        const float4 s = prims[i];
        v[0][0] = s.x; v[0][1] = s.y; v[1][0] = s.z; v[1][1] = s.w;
        nv = 2;
    } else {
        const float4 s0 = prims[3 * i], s1 = prims[3 * i + 1], s2 = prims[3 * i + 2];
        v[0][0] = s0.x; v[0][1] = s0.y; v[0][2] = s0.z;
        v[1][0] = s0.w; v[1][1] = s1.x; v[1][2] = s1.y;
        v[2][0] = s1.z; v[2][1] = s1.w; v[2][2] = s2.x;
        nv = 3;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        lo[a] = v[0][a];
        hi[a] = v[0][a];
        for (int k = 1; k < nv; ++k) { lo[a] = fminf(lo[a], v[k][a]); hi[a] = fmaxf(hi[a], v[k][a]); }
    }
}

// per-block bounds of the primitive centroids: out[block][2D] = (lo, hi)
template <int D>
__global__ __launch_bounds__(256) void lb_bounds_partial(const float4* prims, int n, float* out)
{
    __shared__ float s[256][2 * D];
    float lo[D], hi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        float bl[D], bh[D];
        prim_box<D>(prims, i, bl, bh);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const float c = 0.5f * (bl[a] + bh[a]);
            lo[a] = fminf(lo[a], c);
            hi[a] = fmaxf(hi[a], c);
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) { s[threadIdx.x][a] = lo[a]; s[threadIdx.x][D + a] = hi[a]; }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                s[threadIdx.x][a] = fminf(s[threadIdx.x][a], s[threadIdx.x + w][a]);
                s[threadIdx.x][D + a] = fmaxf(s[threadIdx.x][D + a], s[threadIdx.x + w][D + a]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) out[blockIdx.x * 2 * D + k] = s[0][k];
}

template <int D>
__global__ __launch_bounds__(256) void lb_bounds_final(const float* part, int nblocks, float* out)
{
    __shared__ float s[256][2 * D];
    float lo[D], hi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            lo[a] = fminf(lo[a], part[b * 2 * D + a]);
            hi[a] = fmaxf(hi[a], part[b * 2 * D + D + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) { s[threadIdx.x][a] = lo[a]; s[threadIdx.x][D + a] = hi[a]; }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                s[threadIdx.x][a] = fminf(s[threadIdx.x][a], s[threadIdx.x + w][a]);
                s[threadIdx.x][D + a] = fmaxf(s[threadIdx.x][D + a], s[threadIdx.x + w][D + a]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) out[k] = s[0][k];
}

// spreads the low 10 (3D) or 16 (2D) bits of v to every third / second bit
__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t spread2(uint32_t v)
{
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

template <int D>
__global__ __launch_bounds__(256) void lb_morton(const float4* prims, int n, const float* bounds, uint32_t* keys,
                                                 int32_t* vals)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float bl[D], bh[D];
    prim_box<D>(prims, i, bl, bh);
    const float cells = D == 2 ? 65535.f : 1023.f;
    uint32_t q[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float ext = bounds[D + a] - bounds[a];
        const float t = ext > 0.f ? (0.5f * (bl[a] + bh[a]) - bounds[a]) / ext : 0.f;
        q[a] = (uint32_t)fminf(fmaxf(t * cells, 0.f), cells);
    }
    uint32_t code;
    if (D == 2) code = (spread2(q[0]) << 1) | spread2(q[1]);
    else code = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[D - 1]);
    keys[i] = code;
    vals[i] = i;
}

// common-prefix length of sorted keys i and j; equal keys are told apart by
// their index, and j outside [0, n) gives -1
__device__ __forceinline__ int lb_delta(const uint32_t* k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint32_t a = k[i], b = k[j];
    if (a == b) return 32 + __clz((uint32_t)i ^ (uint32_t)j);
    return __clz(a ^ b);
}

// Binary radix tree: internal nodes 0 .. n-2 (0 is the root), leaf k is node
// n - 1 + k.  Each internal node records its children, its range of sorted
// primitives and is the parent of its children.
__global__ __launch_bounds__(256) void lb_radix_tree(const uint32_t* keys, int n, int32_t* left, int32_t* right,
                                                     int32_t* first, int32_t* last, int32_t* parent)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n - 1) return;
    const int d = lb_delta(keys, n, i, i + 1) - lb_delta(keys, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = lb_delta(keys, n, i, i - d);
    int lmax = 2;
    while (lb_delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (lb_delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = lb_delta(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (lb_delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + (d < 0 ? -1 : 0);
    const int f = i < j ? i : j, lst = i < j ? j : i;
    const int cl = f == gamma ? (n - 1) + gamma : gamma;
    const int cr = lst == gamma + 1 ? (n - 1) + gamma + 1 : gamma + 1;
    left[i] = cl;
    right[i] = cr;
    first[i] = f;
    last[i] = lst;
    parent[cl] = i;
    parent[cr] = i;
    if (i == 0) parent[0] = -1;
}

// Leaf boxes, then boxes up the tree: the second child to reach a node
// (agent-scope acquire-release counter) computes its union.
template <int D>
__global__ __launch_bounds__(256) void lb_boxes(const float4* prims, const int32_t* order, int n, const int32_t* left,
                                                const int32_t* right, const int32_t* parent, uint32_t* arrivals,
                                                float* box)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    int node = (n - 1) + k;
    {
        float lo[D], hi[D];
        prim_box<D>(prims, order[k], lo, hi);
#pragma unroll
        for (int a = 0; a < D; ++a) { box[(int64_t)node * 2 * D + a] = lo[a]; box[(int64_t)node * 2 * D + D + a] = hi[a]; }
    }
    for (;;) {
        const int p = parent[node];
        if (p < 0) break;
        const uint32_t old = __hip_atomic_fetch_add(&arrivals[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0) break;   // the sibling's thread has not arrived yet: it continues
        const int64_t cl = left[p], cr = right[p];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            box[(int64_t)p * 2 * D + a] = fminf(box[cl * 2 * D + a], box[cr * 2 * D + a]);
            box[(int64_t)p * 2 * D + D + a] = fmaxf(box[cl * 2 * D + D + a], box[cr * 2 * D + D + a]);
        }
        node = p;
    }
}

__global__ __launch_bounds__(256) void lb_zero_u32(uint32_t* p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void lb_collapse_init(int32_t* queue, uint32_t* counters)
{
    if (threadIdx.x == 0) {
        queue[0] = 0;       // binary root
        queue[1] = 0;       // four-wide root
        counters[0] = 1;    // four-wide nodes allocated
        counters[1] = 1;    // entries of the current level's queue
        counters[2] = 0;    // entries of the next level's queue
    }
}

__global__ void lb_next_level(uint32_t* counters)
{
    if (threadIdx.x == 0) {
        counters[1] = counters[2];
        counters[2] = 0;
    }
}

// One level of the four-wide collapse: every queue entry (binary node b,
// four-wide node k) writes node k; its inner children get new node indices
// and go to the next level's queue.
template <int D>
__global__ __launch_bounds__(256) void lb_collapse_level(int n, int leaf_size, const int32_t* left,
                                                         const int32_t* right, const int32_t* first,
                                                         const int32_t* last, const float* box, const int32_t* qin,
                                                         int32_t* qout, uint32_t* counters, float4* nodes)
{
    const uint32_t cnt = counters[1];
    const int e = blockIdx.x * 256 + threadIdx.x;
    if ((uint32_t)e >= cnt) return;
    const int b = qin[2 * e], k = qin[2 * e + 1];
    auto size = [&](int c) { return c >= n - 1 ? 1 : last[c] - first[c] + 1; };
    int C[4];
    int nc = 2;
    C[0] = left[b];
    C[1] = right[b];
    while (nc < 4) {
        int best = -1, bsz = leaf_size;
        for (int s = 0; s < nc; ++s) {
            const int sz = size(C[s]);
            if (C[s] < n - 1 && sz > bsz) { best = s; bsz = sz; }
        }
        if (best < 0) break;
        const int c = C[best];
        C[best] = left[c];
        C[nc++] = right[c];
    }
    float lo[D][4], hi[D][4];
    int ref[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ref[s] = kEmptyRef;
#pragma unroll
        for (int a = 0; a < D; ++a) { lo[a][s] = INFINITY; hi[a][s] = -INFINITY; }
        if (s >= nc) continue;
        const int c = C[s];
#pragma unroll
        for (int a = 0; a < D; ++a) { lo[a][s] = box[(int64_t)c * 2 * D + a]; hi[a][s] = box[(int64_t)c * 2 * D + D + a]; }
        const int sz = size(c);
        if (c >= n - 1 || sz <= leaf_size) {
            ref[s] = leaf_ref(c >= n - 1 ? c - (n - 1) : first[c], sz);
        } else {
            const int idx = (int)atomicAdd(&counters[0], 1u);
            const int slot = (int)atomicAdd(&counters[2], 1u);
            qout[2 * slot] = c;
            qout[2 * slot + 1] = idx;
            ref[s] = idx;
        }
    }
    float4* p = nodes + (int64_t)k * Layout4<D>::kDirStride;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        p[a] = make_float4(lo[a][0], lo[a][1], lo[a][2], lo[a][3]);
        p[D + a] = make_float4(hi[a][0], hi[a][1], hi[a][2], hi[a][3]);
    }
    p[2 * D] = make_float4(__int_as_float(ref[0]), __int_as_float(ref[1]), __int_as_float(ref[2]),
                           __int_as_float(ref[3]));
}

// a single primitive: the root holds it as its only (leaf) child
template <int D>
__global__ void lb_single(const float4* prims, float4* nodes, uint32_t* counters, float4* prims_out, int32_t* orig)
{
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int f = 0; f < prim_f4<D>(); ++f) prims_out[f] = prims[f];
    orig[0] = 0;
    float lo[D], hi[D];
    prim_box<D>(prims, 0, lo, hi);
    float4* p = nodes;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        p[a] = make_float4(lo[a], INFINITY, INFINITY, INFINITY);
        p[D + a] = make_float4(hi[a], -INFINITY, -INFINITY, -INFINITY);
    }
    p[2 * D] = make_float4(__int_as_float(leaf_ref(0, 1)), __int_as_float(kEmptyRef), __int_as_float(kEmptyRef),
                           __int_as_float(kEmptyRef));
    counters[0] = 1;
}

// primitives in sorted (leaf) order and their caller indices
template <int D>
__global__ __launch_bounds__(256) void lb_gather(const float4* prims, const int32_t* order, int n, float4* out,
                                                 int32_t* orig)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int src = order[i];
#pragma unroll
    for (int f = 0; f < prim_f4<D>(); ++f) out[(int64_t)prim_f4<D>() * i + f] = prims[(int64_t)prim_f4<D>() * src + f];
    orig[i] = src;
}

template <int D>
__global__ __launch_bounds__(64) void lb_closest(const DevBvh b, const float* pts, int64_t m, float* dist,
                                                 int32_t* prim_out)
{
    extern __shared__ uint2 s_lds[];
    const LdsStack st{&s_lds[threadIdx.x]};
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (i >= m) return;
    float x[D], xbar[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = pts[i * D + a];
    int prim = -1;
    const float best2 = closest_dirichlet<D>(b, x, INFINITY, xbar, &prim, st);
    dist[i] = prim >= 0 ? sqrtf(best2) : INFINITY;
    prim_out[i] = prim >= 0 ? b.orig[prim] : -1;
}

inline int64_t a256(int64_t v) { return (v + 255) & ~int64_t(255); }

struct LbWs {
    uint32_t *keys_in, *keys_out;
    int32_t *vals_in, *vals_out;
    void* sort_tmp;
    size_t sort_bytes;
    int32_t *left, *right, *first, *last, *parent, *queue[2];
    uint32_t *arrivals, *counters;
    float *box, *bparts, *bounds;
};

// workspace carve-up; with base == nullptr only the total is computed
int64_t lb_layout(int dim, int64_t n, uint8_t* base, LbWs* w)
{
    const size_t sort_bytes = (size_t)rs_hist_words(n) * 4;
    const int64_t ni = std::max<int64_t>(n - 1, 1), nt = 2 * n;
    int64_t off = 0;
    auto take = [&](int64_t bytes) { const int64_t o = off; off += a256(bytes); return base ? base + o : nullptr; };
    LbWs t;
    t.keys_in = (uint32_t*)take(n * 4);
    t.keys_out = (uint32_t*)take(n * 4);
    t.vals_in = (int32_t*)take(n * 4);
    t.vals_out = (int32_t*)take(n * 4);
    t.sort_tmp = take((int64_t)sort_bytes);
    t.sort_bytes = sort_bytes;
    t.left = (int32_t*)take(ni * 4);
    t.right = (int32_t*)take(ni * 4);
    t.first = (int32_t*)take(ni * 4);
    t.last = (int32_t*)take(ni * 4);
    t.parent = (int32_t*)take(nt * 4);
    t.queue[0] = (int32_t*)take(2 * ni * 4);
    t.queue[1] = (int32_t*)take(2 * ni * 4);
    t.arrivals = (uint32_t*)take(ni * 4);
    t.counters = (uint32_t*)take(16);
    t.box = (float*)take(nt * 2 * dim * 4);
    t.bparts = (float*)take(kBoundsBlocks * 2 * dim * 4);
    t.bounds = (float*)take(2 * dim * 4);
    if (w) *w = t;
    return off;
}

template <int D>
int lb_build(const float* prims_in, int n, int leaf_size, float* nodes_out, float* prims_out, int32_t* orig,
             int32_t* n_nodes, int32_t* levels, const LbWs& w, hipStream_t s)
{
    const float4* P = (const float4*)prims_in;
    float4* N = (float4*)nodes_out;
    const int g256 = (n + 255) / 256;
    if (n == 1) {
        hipLaunchKernelGGL(lb_single<D>, dim3(1), dim3(64), 0, s, P, N, w.counters, (float4*)prims_out, orig);
        *n_nodes = 1;
        *levels = 1;
        return hipStreamSynchronize(s) == hipSuccess ? WOST_OK : WOST_EHIP;
    }
    const int pb = std::min(kBoundsBlocks, g256);
    hipLaunchKernelGGL(lb_bounds_partial<D>, dim3(pb), dim3(256), 0, s, P, n, w.bparts);
    hipLaunchKernelGGL(lb_bounds_final<D>, dim3(1), dim3(256), 0, s, w.bparts, pb, w.bounds);
    hipLaunchKernelGGL(lb_morton<D>, dim3(g256), dim3(256), 0, s, P, n, w.bounds, w.keys_in, w.vals_in);
    if (rs_sort_pairs(w.keys_in, w.vals_in, w.keys_out, w.vals_out, n, 32, (uint32_t*)w.sort_tmp, s) != WOST_OK) {
        set_error("wost_lbvh_build: radix sort failed: %s", hipGetErrorString(hipGetLastError()));
        return WOST_EHIP;
    }
    const int gi = (n - 1 + 255) / 256;
    hipLaunchKernelGGL(lb_radix_tree, dim3(gi), dim3(256), 0, s, w.keys_out, n, w.left, w.right, w.first, w.last,
                       w.parent);
    hipLaunchKernelGGL(lb_zero_u32, dim3(gi), dim3(256), 0, s, w.arrivals, n - 1);
    hipLaunchKernelGGL(lb_boxes<D>, dim3(g256), dim3(256), 0, s, P, w.vals_out, n, w.left, w.right, w.parent,
                       w.arrivals, w.box);
    hipLaunchKernelGGL(lb_collapse_init, dim3(1), dim3(64), 0, s, w.queue[0], w.counters);
    // every level takes at least one binary level, and a binary path is at
    // most 64 nodes long (32 key bits + 32 index bits)
    int lv = 0;
    for (; lv < kMaxLbvhLevels; ++lv) {
        uint32_t cnt = 0;
        if (hipMemcpyAsync(&cnt, w.counters + 1, sizeof(cnt), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("wost_lbvh_build: %s", hipGetErrorString(hipGetLastError()));
            return WOST_EHIP;
        }
        if (cnt == 0) break;
        hipLaunchKernelGGL(lb_collapse_level<D>, dim3((cnt + 255) / 256), dim3(256), 0, s, n, leaf_size, w.left,
                           w.right, w.first, w.last, w.box, w.queue[lv & 1], w.queue[(lv + 1) & 1], w.counters, N);
        hipLaunchKernelGGL(lb_next_level, dim3(1), dim3(64), 0, s, w.counters);
    }
    if (lv == kMaxLbvhLevels) {
        set_error("wost_lbvh_build: more than %d four-wide levels", kMaxLbvhLevels);
        return WOST_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(lb_gather<D>, dim3(g256), dim3(256), 0, s, P, w.vals_out, n, (float4*)prims_out, orig);
    uint32_t nn = 0;
    if (hipMemcpyAsync(&nn, w.counters, sizeof(nn), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("wost_lbvh_build: %s", hipGetErrorString(hipGetLastError()));
        return WOST_EHIP;
    }
    *n_nodes = (int32_t)nn;
    *levels = lv;
    return WOST_OK;
}

}  // namespace
}  // namespace wost

using namespace wost;

extern "C" int wost_lbvh_sizes(int32_t dim, int64_t n, int64_t* node_bytes, int64_t* prim_bytes, int64_t* ws_bytes)
{
    if ((dim != 2 && dim != 3) || n < 1 || n > kMaxLeafFirst || !node_bytes || !prim_bytes || !ws_bytes) {
        set_error("wost_lbvh_sizes: dim 2 or 3, 1 <= n < 2^25 - 64, non-NULL outputs");
        return WOST_EINVAL;
    }
    const int stride = 2 * dim + 1;
    *node_bytes = std::max<int64_t>(n - 1, 1) * stride * 16;
    *prim_bytes = n * (dim == 2 ? 1 : 3) * 16;
    *ws_bytes = lb_layout(dim, n, nullptr, nullptr);
    return WOST_OK;
}

extern "C" int wost_lbvh_build(int32_t dim, const float* prims, int64_t n, int32_t leaf_size, float* nodes,
                               float* prims_sorted, int32_t* orig, int32_t* n_nodes, int32_t* levels,
                               void* workspace, int64_t ws_bytes, void* stream)
{
    int64_t nb = 0, pbytes = 0, need = 0;
    if (wost_lbvh_sizes(dim, n, &nb, &pbytes, &need) != WOST_OK) return WOST_EINVAL;
    if (!prims || !nodes || !prims_sorted || !orig || !n_nodes || !levels || !workspace) {
        set_error("wost_lbvh_build: NULL argument");
        return WOST_EINVAL;
    }
    if (leaf_size < 1 || leaf_size > kLeafMax) { set_error("wost_lbvh_build: leaf_size in [1, 64]"); return WOST_EINVAL; }
    if (ws_bytes < need) { set_error("wost_lbvh_build: workspace %lld < %lld bytes", (long long)ws_bytes, (long long)need); return WOST_ESIZE; }
    if (((uintptr_t)workspace & 255) || ((uintptr_t)prims & 15) || ((uintptr_t)nodes & 15) || ((uintptr_t)prims_sorted & 15)) {
        set_error("wost_lbvh_build: workspace must be 256-byte aligned, prims and nodes 16-byte aligned");
        return WOST_EINVAL;
    }
    LbWs w;
    lb_layout(dim, n, (uint8_t*)workspace, &w);
    hipStream_t s = (hipStream_t)stream;
    const int rc = dim == 2 ? lb_build<2>(prims, (int)n, leaf_size, nodes, prims_sorted, orig, n_nodes, levels, w, s)
                            : lb_build<3>(prims, (int)n, leaf_size, nodes, prims_sorted, orig, n_nodes, levels, w, s);
    if (rc != WOST_OK) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_lbvh_build: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}

extern "C" int wost_lbvh_closest(int32_t dim, const float* nodes, int32_t n_nodes, const float* prims_sorted,
                                 const int32_t* orig, int32_t n_prims, int32_t levels, const float* pts, int64_t m,
                                 float* dist, int32_t* prim, void* stream)
{
    if ((dim != 2 && dim != 3) || !nodes || !prims_sorted || !orig || n_nodes < 1 || n_prims < 1 || levels < 1 ||
        m < 0 || (m > 0 && (!pts || !dist || !prim))) {
        set_error("wost_lbvh_closest: bad arguments");
        return WOST_EINVAL;
    }
    // a traversal defers at most three children per level of its path
    const int64_t entries = 3 * ((int64_t)levels - 1) + 1;
    const size_t lds = sizeof(uint2) * (size_t)entries * kWave;
    if (lds > 64 * 1024) { set_error("wost_lbvh_closest: %d levels need more LDS than a workgroup has", levels); return WOST_EUNSUPPORTED; }
    if (m == 0) return WOST_OK;
    DevBvh b{};
    memset(&b, 0, sizeof(b));
    b.nodes = (const float4*)nodes;
    b.prims = (const float4*)prims_sorted;
    b.orig = orig;
    b.n_nodes = n_nodes;
    b.n_prims = n_prims;
    hipStream_t s = (hipStream_t)stream;
    const int grid = (int)((m + 63) / 64);
    if (dim == 2) hipLaunchKernelGGL(lb_closest<2>, dim3(grid), dim3(64), lds, s, b, pts, m, dist, prim);
    else hipLaunchKernelGGL(lb_closest<3>, dim3(grid), dim3(64), lds, s, b, pts, m, dist, prim);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error("wost_lbvh_closest: launch failed: %s", hipGetErrorString(e)); return WOST_EHIP; }
    return WOST_OK;
}
