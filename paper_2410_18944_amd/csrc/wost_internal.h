// Internal layout shared by the host builder and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wost.h"

namespace wost {

constexpr int kMaxStack = 24;      // traversal stack entries per lane (LDS)
constexpr int kMaxDepth = kMaxStack - 1;
constexpr int kWave = 64;

// Binary BVH node holding both children's boxes, so one fetch decides the
// visit order.  ch = (c0, n0, c1, n1): n_i > 0 -> leaf with primitives
// [c_i, c_i + n_i); n_i == 0 && c_i >= 0 -> inner node c_i; c_i < 0 -> empty.
// aux_i: Neumann hierarchy -> (subtree measure, 0, 0, 0);
//        silhouette hierarchy -> (cone axis xyz (2D: xy,0), half angle).
struct alignas(16) Node2 {
    float4 b0;      // lo.x lo.y hi.x hi.y
    float4 b1;
    int4 ch;
    float4 aux0;
    float4 aux1;
};
struct alignas(16) Node3 {
    float4 b0a;     // lo0.xyz hi0.x
    float4 b0b;     // hi0.yz lo1.xy
    float4 b1b;     // lo1.z hi1.xyz
    int4 ch;
    float4 aux0;
    float4 aux1;
};

template <int D> struct NodeT;
template <> struct NodeT<2> { using type = Node2; };
template <> struct NodeT<3> { using type = Node3; };

// Primitive records.
//  2D segment: float4 (a.x, a.y, b.x, b.y)
//  3D triangle: 3 x float4: (a.xyz, b.x) (b.yz, c.xy) (c.z, pad...)
//  Neumann extra per primitive: float4 (n_out.xyz (2D: xy,0), measure)
//  Silhouette 2D: 2 x float4: (v.xy, n1.xy) (n2.xy, q1, q2)
//  Silhouette 3D: 4 x float4: (a.xyz, b.x) (b.yz, n1.xy) (n1.z, n2.xyz) (q1, q2, 0, 0)
//                 n1, n2 inward normals of the adjacent Neumann primitives,
//                 q1, q2 their internal Neumann ids as int bit patterns
//                 (q2 = -1: boundary feature with a single Neumann neighbour)
struct DevBvh {
    const void* nodes;      // NodeT<D>[n_nodes]
    const float4* prims;    // prim records
    const float4* pextra;   // Neumann per-primitive normal + measure (or null)
    const int32_t* orig;    // internal primitive id -> caller primitive index
    int32_t n_nodes;
    int32_t n_prims;
};

struct DevGeom {
    DevBvh dir;             // Dirichlet primitives
    DevBvh neu;             // Neumann primitives
    DevBvh sil;             // Neumann silhouette candidates
    int32_t dim;
    float diag;             // AABB diagonal L
    float tau;              // facing / self-intersection tolerance (1e-6 L)
    float lo[3], hi[3];
};

struct FieldDev {
    int32_t kind;
    int32_t n;
    float p[WOST_MAX_GAUSS * 5];
};

}  // namespace wost

// Opaque handle (host side).
struct wost_geom {
    int32_t dim = 0;
    int64_t n_dir = 0, n_neu = 0, n_sil = 0;
    int32_t max_depth = 0;
    double diag = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    // host image of the device buffer and section offsets (bytes)
    uint8_t* image = nullptr;
    int64_t bytes = 0;
    struct Sec { int64_t nodes, prims, pextra, orig; int32_t n_nodes, n_prims; } sec[3];
    void* dev = nullptr;    // caller buffer after upload
    int32_t* orig_host = nullptr;    // concatenated: dir, neu prims -> caller ids
    wost::DevGeom devgeom() const;
};

namespace wost {
void set_error(const char* fmt, ...);
}  // namespace wost
