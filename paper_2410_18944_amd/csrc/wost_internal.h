// Internal layout shared by the host builder and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/wost.h"

namespace wost {

constexpr int kMaxStack = 40;      // traversal stack entries per lane (LDS)
constexpr int kWave = 64;

// Four-wide BVH node: the four children of a node are stored as structure of
// arrays, one float4 per coordinate, so a single node fetch tests all four.
// Node i of a hierarchy is the run of float4 at nodes + i * stride:
//   [0, D)       lo.x, lo.y (, lo.z) of children 0..3
//   [D, 2D)      hi.x, hi.y (, hi.z)
//   2D           int4 child references (bit patterns):
//                  >= 0          inner child: node index
//                  kEmptyRef     no child (its box is empty and never tested)
//                  other < 0     leaf: -1 - (first * 64 + count - 1),
//                                primitives [first, first + count), count <= 64
//   2D + 1 ...   per-hierarchy child data:
//                  Dirichlet     none                          stride 2D + 1
//                  Neumann       subtree measure (1 float4)    stride 2D + 2
//                  silhouettes   normal cone axis x, y (, z), cos
//                                of its half-angle, and the convex
//                                piece all its candidates are interior
//                                to (int bits, -1 for none)    stride 3D + 3
constexpr int32_t kEmptyRef = (int32_t)0x80000000;
constexpr int kLeafMax = 64;
constexpr int64_t kMaxLeafFirst = (1ll << 25) - kLeafMax;   // first < this

template <int D> struct Layout4 {
    static constexpr int kRef = 2 * D;
    static constexpr int kAux = 2 * D + 1;
    static constexpr int kDirStride = 2 * D + 1;
    static constexpr int kNeuStride = 2 * D + 2;
    static constexpr int kSilStride = 3 * D + 3;
    static constexpr int kPiece = 3 * D + 2;
};

__host__ __device__ inline int32_t leaf_ref(int32_t first, int32_t count) { return -1 - (first * kLeafMax + count - 1); }
__host__ __device__ inline int32_t leaf_first(int32_t ref) { return (-1 - ref) / kLeafMax; }
__host__ __device__ inline int32_t leaf_count(int32_t ref) { return (-1 - ref) % kLeafMax + 1; }

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
    const float4* nodes;    // n_nodes four-wide nodes (layout above)
    const float4* prims;    // prim records
    const float4* pextra;   // Neumann per-primitive normal + measure (or null)
    const int32_t* orig;    // internal primitive id -> caller primitive index
    const int32_t* piece;   // silhouettes: convex piece of each Neumann primitive
                            // (internal Neumann id), -1 for none; else null
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
    const int32_t* neu_id;  // caller primitive index -> internal Neumann id (-1: Dirichlet)
    int64_t n_caller;       // caller primitives
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
    int32_t max_depth = 0;          // deepest binary split level (reported)
    int32_t stack_entries = 0;      // traversal stack entries a lane needs
    double diag = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    // host image of the device buffer and section offsets (bytes)
    uint8_t* image = nullptr;
    int64_t bytes = 0;
    struct Sec { int64_t nodes, prims, pextra, orig, piece; int32_t n_nodes, n_prims; } sec[3];
    int64_t off_neu_id = -1;        // caller id -> internal Neumann id table
    int64_t n_caller = 0;
    void* dev = nullptr;    // caller buffer after upload
    int32_t* orig_host = nullptr;    // concatenated: dir, neu prims -> caller ids
    // a Dirichlet hierarchy built on the device over the same primitives,
    // used in place of the image's Dirichlet section when nodes is set
    struct DirDev {
        const void* nodes = nullptr;
        const void* prims = nullptr;
        const int32_t* orig = nullptr;
        int32_t n_nodes = 0, n_prims = 0, stack = 0;
    } dir_dev;
    // a geometry built on the device: the image's arrays as they lie in the
    // build workspace, copied to their offsets by wost_geom_upload
    struct Staged { const void* src; int64_t off, bytes; };
    std::vector<Staged> staged;
    wost::DevGeom devgeom() const;
    // traversal stack entries a lane needs with the hierarchies in use
    int32_t stack_need() const { return dir_dev.nodes && dir_dev.stack > stack_entries ? dir_dev.stack : stack_entries; }
};

namespace wost {
void set_error(const char* fmt, ...);
}  // namespace wost
