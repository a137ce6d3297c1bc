/*
 * wost.h -- C ABI of the MI355X (gfx950) guided walk-on-stars library.
 *
 * The library estimates the solution u of the mixed Poisson problem
 *     Laplacian u = f  in the domain,  u = g on the Dirichlet part,
 *     du/dn = h on the Neumann part
 * (paper Sec. 3.1, equation "linear_elliptic") at query points by the walk on
 * stars estimator (Sec. 3.2, equation "wost_estm"), with the recursive term's
 * direction drawn uniformly or from a learned von Mises-Fisher mixture
 * combined with uniform sampling by one-sample MIS (Secs. 4.1-4.4).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Status: every int-returning call returns WOST_OK (0) or a negative
 *   WOST_E* code; wost_last_error() then holds a thread-local message.
 *   Nothing throws across the ABI, nothing aborts or exits.
 * - Memory: device buffers are allocated by the CALLER (e.g. as torch
 *   tensors) and passed as raw device pointers; the library never allocates
 *   device memory.  Size queries (*_bytes) tell the caller what to allocate.
 *   Host pointers are only read during the call unless stated otherwise.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *   stream).  Launches are asynchronous on that stream; nothing synchronises
 *   except wost_build_bvh (host-only), wost_build_bvh_device and wost_geom_upload
 *   (which synchronise the stream they are given).
 * - Layouts: points and directions are row-major [n][dim] float32 (AoS).
 * - Handles are not thread-safe; distinct handles may be used concurrently.
 */
#ifndef WOST_H
#define WOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define WOST_OK 0
#define WOST_EINVAL (-1)        /* invalid argument (NULL, out-of-range, bad shape)   */
#define WOST_ESIZE (-2)         /* caller buffer too small                             */
#define WOST_EHIP (-3)          /* a HIP runtime call failed                           */
#define WOST_ESTATE (-4)        /* handle in the wrong state (e.g. not uploaded/bound) */
#define WOST_EUNSUPPORTED (-5)  /* valid but unsupported configuration                 */

/* Thread-local description of the last error on this thread ("" if none). */
const char* wost_last_error(void);

/* Opaque handles. */
typedef struct wost_geom wost_geom;     /* boundary hierarchies          */
typedef struct wost_guide wost_guide;   /* neural guiding field          */

/* ------------------------------------------------------------ fields
 * Analytic fields for the boundary data g, h and the source f.
 *   WOST_FIELD_ZERO        0
 *   WOST_FIELD_CONST       params[0]
 *   WOST_FIELD_EXP_SIN     e^x sin y
 *   WOST_FIELD_RE_Z3       Re z^3 = x^3 - 3 x y^2
 *   WOST_FIELD_X2_MINUS_Y2 x^2 - y^2
 *   WOST_FIELD_R2          |x|^2
 *   WOST_FIELD_GAUSS_SUM   sum_j a_j exp(-|x - c_j|^2 / (2 s_j^2)),
 *                          params = n rows of (a_j, s_j, c_j[dim]); n <= 32
 * For the Neumann data h, a CONST kind is the outward flux du/dn_out itself and
 * any other kind phi means h = grad(phi) . n_out (outward normal derivative).
 * params is a HOST pointer read during the call. */
#define WOST_FIELD_ZERO 0
#define WOST_FIELD_CONST 1
#define WOST_FIELD_EXP_SIN 2
#define WOST_FIELD_RE_Z3 3
#define WOST_FIELD_X2_MINUS_Y2 4
#define WOST_FIELD_R2 5
#define WOST_FIELD_GAUSS_SUM 6
#define WOST_MAX_GAUSS 32

typedef struct {
    int32_t kind;
    int32_t n;              /* number of parameter rows (GAUSS_SUM) or values */
    const float* params;    /* host */
} wost_field;

/* ------------------------------------------------------------ geometry
 * wost_build_bvh: host-side build of the boundary representation.
 *   dim      2 (polyline segments) or 3 (triangles)
 *   verts    host float32 [n_verts][dim]
 *   prims    host int32 [n_prims][dim] vertex ids.  Winding: in 2D the domain
 *            lies to the LEFT of each directed segment a->b; in 3D (b-a)x(c-a)
 *            points OUT of the domain.
 *   bc       host uint8 [n_prims]: 0 = Dirichlet, 1 = Neumann
 *   opts     NULL for defaults
 * Builds bounding volume hierarchies over the Dirichlet primitives (closest
 * point, Sec. 3.2), the Neumann primitives (rays, visibility, Neumann-term
 * sampling) and the Neumann silhouette candidates -- vertices in 2D, edges in
 * 3D -- with normal cones (closest silhouette; the star radius of Sec. 3.2).
 * Degenerate primitives (zero length / area) and out-of-range vertex ids
 * give WOST_EINVAL.  On success *out owns a host image of the device layout. */
typedef struct {
    int32_t leaf_size;      /* max primitives per leaf (default 4, 1..64)             */
    int32_t brute_force;    /* 1: exhaustive queries: leaves of 64 primitives whose
                               boxes cover the whole hierarchy, no cone culling      */
} wost_build_opts;

int wost_build_bvh(int32_t dim, const float* verts, int64_t n_verts, const int32_t* prims,
                   int64_t n_prims, const uint8_t* bc, const wost_build_opts* opts, wost_geom** out);
/* wost_build_bvh_device: the same build from device inputs, run on the GPU
 * (the query library's hierarchies built in parallel, Sec. 5.3), giving the
 * image wost_build_bvh gives byte for byte.
 *   verts, prims, bc   device arrays, layouts as for wost_build_bvh
 *   opts               NULL or leaf_size in 1..64; brute_force gives
 *                      WOST_EUNSUPPORTED
 *   workspace          device, 256-byte aligned, >= the bytes that
 *                      wost_build_bvh_device_workspace reports (an upper
 *                      bound from n_prims and leaf_size: about 0.7 KB per
 *                      primitive in 2D and 1 KB in 3D)
 *   stream             the build's kernels and copies; the call synchronises
 *                      it several times and returns with it idle
 * Invalid input gives WOST_EINVAL with the first offending vertex or
 * primitive in the host builder's order; sets beyond 2^25 - 64 primitives or
 * hierarchies deeper than the traversal stack give WOST_EUNSUPPORTED.  The
 * built image stays in the workspace: wost_geom_upload copies it into the
 * caller's buffer, so the workspace must stay untouched until that upload
 * has returned; it may be freed or reused afterwards.  wost_geom_info and
 * wost_geom_prim_index work on the handle at once. */
int wost_build_bvh_device_workspace(int32_t dim, int64_t n_verts, int64_t n_prims, const wost_build_opts* opts,
                                    int64_t* ws_bytes);
int wost_build_bvh_device(int32_t dim, const float* verts, int64_t n_verts, const int32_t* prims, int64_t n_prims,
                          const uint8_t* bc, const wost_build_opts* opts, void* workspace, int64_t ws_bytes,
                          void* stream, wost_geom** out);
/* Bytes of device memory the geometry needs (256-byte aligned base required). */
int64_t wost_geom_device_bytes(const wost_geom* geom);
/* Copy the geometry into the caller-owned device buffer `dev_buf` (>= bytes)
 * on `stream`, and synchronise that stream: host to device for a host build,
 * device to device (padding zeroed) for a device build.  The buffer must
 * outlive every call that uses `geom`.  Re-uploading to another buffer is
 * allowed. */
int wost_geom_upload(wost_geom* geom, void* dev_buf, int64_t bytes, void* stream);
/* Scene statistics: out[0..7] = dim, n_dirichlet, n_neumann, n_silhouette,
 * deepest binary split level, AABB diagonal, bytes, traversal stack entries
 * per lane (the hierarchies are stored four-wide: every node holds the
 * children of a binary node with inner children replaced by their own). */
int wost_geom_info(const wost_geom* geom, double* out8);
/* Map a library-internal primitive id (as returned by wost_query) to the
 * caller's primitive index; returns -1 if out of range. */
int64_t wost_geom_prim_index(const wost_geom* geom, int32_t internal_id);
void wost_geom_free(wost_geom* geom);

/* Batched geometric queries of the walk (for inspection and parity tests).
 *   pts          device [n][dim]
 *   on_prim      device [n] or NULL: caller index of the Neumann primitive each
 *                point lies on (-1 = none); such a primitive faces its point
 *                from the front in the silhouette query, as for a walker
 *                standing on it (Sec. 3.2)
 *   d_dir, xbar  device [n], [n][dim]: distance to / closest point on the
 *                Dirichlet boundary (Sec. 3.2 epsilon-shell test); NULL to skip
 *   d_sil        device [n]: distance to the closest Neumann silhouette point
 *                seen from pts (the second bound of the star radius); NULL to skip
 *   ray_dir, ray_tmax  device [n][dim] unit directions, [n] max distance; with
 *                ray_t [n] and ray_prim [n] (caller primitive index, -1 = miss)
 *                gives the first Neumann hit in (tau, tmax); NULL to skip.
 * Missing results are +inf. */
int wost_query(const wost_geom* geom, const float* pts, int64_t n, const int32_t* on_prim,
               float* d_dir, float* xbar, float* d_sil, const float* ray_dir, const float* ray_tmax,
               float* ray_t, int32_t* ray_prim, void* stream);

/* The Neumann-sample step of a walk for given states (for parity tests of
 * the Neumann contribution, Sec. 3.2 eq. wost_estm): one primitive meeting
 * the ball B(x, r) is chosen by a descent of the Neumann hierarchy (children
 * in proportion to their subtree measure, then a leaf primitive in proportion
 * to its measure among those meeting the ball), a point z uniform on it, and
 * z is accepted if |z - x| < r, it does not lie behind the walker's tangent
 * plane (points on a Neumann primitive), and it is visible from the walker's
 * ray origin.  The walk then scores G_r(|z - x|) h(z) |q| / prob / alpha.
 *   pts       device [n][dim]; on_prim device [n] or NULL (as wost_query)
 *   radius    device [n] star radii r
 *   uniforms  device [n][3] numbers in [0, 1): the descent's uniform and the
 *             two that place z on the primitive
 *   prim      device [n] caller index of the chosen primitive (-1: none)
 *   prob      device [n] probability with which it was chosen
 *   z         device [n][dim] the point (+inf if none)
 *   accepted  device [n] 1 if z passed the checks above, else 0 */
int wost_neumann_sample(const wost_geom* geom, const float* pts, int64_t n, const int32_t* on_prim,
                        const float* radius, const float* uniforms, int32_t* prim, float* prob, float* z,
                        int32_t* accepted, void* stream);

/* ------------------------------------------------------------ problem + solve */
#define WOST_SAMPLING_UNIFORM 0      /* original WoSt: uniform directions (c = 0)       */
#define WOST_SAMPLING_MIS_LEARNED 1  /* MIS with the guide's learned c(x) (Sec. 4.4)    */
#define WOST_SAMPLING_MIS_FIXED 2    /* MIS with c = c_fixed                             */
#define WOST_SAMPLING_GUIDED_ONLY 3  /* c = 1                                            */

typedef struct {
    wost_field g;           /* Dirichlet value, evaluated at the closest point          */
    wost_field h;           /* Neumann data (outward derivative), see fields above       */
    wost_field f;           /* source with Laplacian u = f                               */
    float eps;              /* epsilon-shell width (Sec. 3.2)                            */
    float r_min;            /* lower clamp of the star radius (0 = use eps)              */
    int32_t max_steps;      /* step cap; the walk then takes g at the closest point      */
    int32_t rr_start;       /* Russian roulette from this step on (Sec. 6.1: 128)       */
    float rr_q;             /* roulette survival probability                             */
    int32_t sampling;       /* WOST_SAMPLING_*                                           */
    float c_fixed;          /* selection probability for WOST_SAMPLING_MIS_FIXED         */
    int32_t reflect;        /* guided draws into the wall at a Neumann point:
                               1 = reflected about the tangent plane (Sec. 4.3),
                               0 = wasted (the walk ends there with zero
                               recursive term; the reflection ablation of
                               Sec. 6).  Guided solves require it to equal the
                               guide's setting (wost_guide_set_reflect), else
                               WOST_EINVAL.  Uniform draws always use the valid
                               half                                              */
} wost_problem;

/* Training records written by guided walks (one per drawn direction), in a
 * caller-owned device buffer of `capacity` rows, structure-of-arrays:
 * field f of row i is at data[f * capacity + i].  Fields (dim = d):
 *   0..d-1     x_k           walk location
 *   d..2d-1    nu_k          drawn direction (after reflection, if on;
 *                            wasted draws write no record)
 *   2d..3d-1   n_k           unit normal on the walk's side if x_k is on the
 *                            Neumann boundary, else 0
 *   3d         p_sample      MIS pdf of nu_k at draw time
 *   3d+1       prefix        sum of T_j (N_j + S_j) over j <= k
 *   3d+2       T_next        throughput T_{k+1} = T_k w_k (roulette folded in)
 *   3d+3       slot          walk slot (int32 bits) in the call's walk order
 *   3d+4       p_t           training target |V_{k+1}|, filled by
 *                            wost_tail_pass (Sec. 4.1 target distribution)
 * `count` is a device int64 counter of rows appended (may exceed capacity:
 * rows beyond capacity are dropped and counted in dev_counters[6]). */
#define WOST_REC_FIELDS(d) (3 * (d) + 5)
typedef struct {
    float* data;            /* device [WOST_REC_FIELDS(d)][capacity] */
    int64_t capacity;
    int64_t* count;         /* device */
} wost_records;

/* Workspace bytes needed by wost_solve for n_points x wpp walks: a walk
 * counter, one float per walk, and the walk pools of the persistent kernel
 * (per wave, a structure of arrays of up to `slots_per_wave` walks plus its
 * work lists; see wost_set_walk_pool).  The figure depends on the device's
 * compute-unit count and the pool setting at the time of the call. */
int64_t wost_solve_workspace_bytes(const wost_geom* geom, int64_t n_points, int32_t wpp);

/* Walk-on-stars solve (Sec. 3.2 estimator; Sec. 4 guided directions).
 *   pts         device [n_points][dim] query points
 *   wpp         walks per point; walk (p, j) uses Philox4x32-10 keyed by `seed`
 *               with counter (p, walk_offset + j, step, block), so results do
 *               not depend on how walks are split over calls
 *   guide       NULL iff problem->sampling == WOST_SAMPLING_UNIFORM
 *   sum, sum_sq, count   device [n_points] float64 / int64, ACCUMULATED (+=)
 *               with the per-point sum of walk values, of squares, and walks
 *   walk_value  device [n_points*wpp] float32 or NULL: per-walk estimate,
 *               index p*wpp + j
 *   walk_steps  device [n_points*wpp] int32 or NULL: stars visited per walk
 *   rec         NULL, or training records to append (guided runs)
 *   workspace   device, >= wost_solve_workspace_bytes
 *   dev_counters device uint64 [8], ACCUMULATED: steps, walks, truncated
 *               (step cap), roulette kills, non-finite weights, records,
 *               records dropped, 0.
 * Every walk step visits one star: closest Dirichlet point (epsilon-shell
 * termination, Sec. 3.2), closest Neumann silhouette -> radius r, Neumann
 * and source contributions, direction draw, first hit inside the star. */
int wost_solve(const wost_geom* geom, const wost_problem* problem, const float* pts,
               int64_t n_points, int32_t wpp, uint64_t seed, uint64_t walk_offset,
               const wost_guide* guide, double* sum, double* sum_sq, int64_t* count,
               float* walk_value, int32_t* walk_steps, const wost_records* rec, void* workspace,
               int64_t ws_bytes, uint64_t* dev_counters, void* stream);

/* The same solve organised as the paper's GPU system (Sec. 5.1; Sec. 5.2
 * "System Integration"): the state of every walk of the call lives in the
 * workspace, and each step of all live walks is a sequence of kernels, one
 * per stage (closest Dirichlet point, silhouette and radius, guided direction
 * batched over all stepping walks, Neumann sample and its visibility, source
 * point and its visibility, first hit, update), over queues of walk ids that
 * each stage compacts for the next.  With two streams set
 * (wost_set_wavefront_streams), guided solves split the walks into two
 * halves and run the network of one half on a second stream (created by the
 * library once per device, default priority) while the caller's stream runs
 * the geometric stages of the other half.  Arguments, outputs and errors as
 * wost_solve; walks use the same random words and traversal code, so per-walk
 * values and step counts agree with wost_solve's.  Unlike wost_solve it
 * waits on `stream`: the host reads the live-walk count back every eight
 * steps and stops when it reaches zero.  Traversal-cost counters
 * (wost_set_cost_counters) are not supported (WOST_EUNSUPPORTED).  Kept as
 * the baseline the persistent kernel is measured against. */
/* Streams of guided wavefront solves: 1 (default; every stage on the
 * caller's stream) or 2 (the network on a second stream, overlapping the
 * geometric stages of the other half of the walks, as in Sec. 5.2 "System
 * Integration").  Process wide; results do not depend on it.  Other values:
 * WOST_EINVAL. */
int wost_set_wavefront_streams(int32_t n_streams);
int64_t wost_solve_wavefront_workspace_bytes(const wost_geom* geom, int64_t n_points, int32_t wpp);
int wost_solve_wavefront(const wost_geom* geom, const wost_problem* problem, const float* pts, int64_t n_points,
                         int32_t wpp, uint64_t seed, uint64_t walk_offset, const wost_guide* guide, double* sum,
                         double* sum_sq, int64_t* count, float* walk_value, int32_t* walk_steps,
                         const wost_records* rec, void* workspace, int64_t ws_bytes, uint64_t* dev_counters,
                         void* stream);

/* ------------------------------------------------------------ guide
 * The neural field of Sec. 5.2: a multi-resolution grid (hashed where a
 * level's dense lattice exceeds the table) followed by a bias-free ReLU MLP
 * whose K*(dim+2)+1 outputs are mapped by Tab. "reg_map" to K vMF lobes
 * (mu, kappa, lambda) and the MIS selection probability c (Sec. 4.4). */
typedef struct {
    int32_t dim;            /* 2 or 3                                         */
    int32_t levels;         /* L                                              */
    int32_t feats;          /* F (must be 2)                                  */
    int32_t log2_table;     /* log2 of entries per level                      */
    int32_t n_min, n_max;   /* coarsest / finest lattice resolution           */
    int32_t hidden;         /* width (must be 64)                             */
    int32_t n_hidden;       /* hidden layers (1..4)                           */
    int32_t K;              /* lobes (1..16)                                  */
    float aabb_lo[3];       /* input normalisation box                        */
    float aabb_hi[3];
} wost_guide_config;

int wost_guide_create(const wost_guide_config* cfg, wost_guide** out);
/* Number of trainable parameters P (grid entries * F + MLP weights).  The
 * flat float32 layout is: grid [L][T][F], then each layer's weight matrix
 * row-major [in][out] (first layer in = L*F, hidden width 64, last out =
 * K*(dim+2)+1; per lobe (mu'_1..mu'_dim, kappa', lambda'), then c'). */
int64_t wost_guide_param_count(const wost_guide* g);
/* Sample reflection at Neumann points (Sec. 4.3), default 1.  With 0, the
 * guided branch of a draw at a Neumann point keeps the plain mixture: a draw
 * with nu . n <= 0 is wasted, and p_g on the valid half is the mixture itself
 * (the "without reflection" variant of the ablation in Sec. 6).  The setting
 * is read by wost_guide_sample, by the training loss (which p_g a Neumann
 * record is scored with) and checked against wost_problem.reflect by
 * wost_solve.  reflect must be 0 or 1, else WOST_EINVAL. */
int wost_guide_set_reflect(wost_guide* g, int32_t reflect);
/* The current setting (0 or 1), -1 for a NULL handle. */
int32_t wost_guide_get_reflect(const wost_guide* g);
/* Bytes of the half-precision shadow used by inference (grid entries in the
 * same order, MLP weights re-arranged into MFMA operand fragments). */
int64_t wost_guide_shadow_bytes(const wost_guide* g);
/* Bind caller-owned device storage: master float32 [P], shadow
 * [wost_guide_shadow_bytes] (16-byte aligned, else WOST_EINVAL), Adam moments
 * m, v float32 [P], gradient float32 [P].  Any of adam_m/adam_v/grad may be
 * NULL for inference-only use.  Pointers must stay valid while the guide is used. */
int wost_guide_bind(wost_guide* g, float* master, void* shadow_f16, float* adam_m, float* adam_v,
                    float* grad);
/* Seeded initialisation of master, shadow, and zeroing of Adam state:
 * grid U(-1e-4, 1e-4), MLP He-uniform. */
int wost_guide_init(wost_guide* g, uint64_t seed, void* stream);
/* Refresh the fp16 shadow from the float32 master parameters. */
int wost_guide_sync_shadow(wost_guide* g, void* stream);
/* Raw network outputs (before the normalisation mapping) at n points:
 * pts device [n][dim], out_raw device [n][K*(dim+2)+1]. */
int wost_guide_infer(const wost_guide* g, const float* pts, int64_t n, float* out_raw, void* stream);
/* One MIS direction draw per point, exactly as the walk draws it at step 0
 * of walk (i, walk_index) with Philox key `seed`: pts device [n][dim];
 * normals device [n][dim] or NULL -- a nonzero row marks a point on the
 * Neumann boundary with that unit normal on the walk's side (draws are then
 * reflected into the valid half, Sec. 4.3, if the guide's reflection setting
 * is on); sampling is a guided WOST_SAMPLING_* mode.  Outputs: out_nu
 * [n][dim], out_pdf [n] = the MIS pdf c p_g + (1 - c) p_u of the returned
 * direction (Sec. 4.4), or -1 for a wasted draw (reflection off: a guided
 * draw with nu . n <= 0, returned unreflected). */
int wost_guide_sample(const wost_guide* g, int32_t sampling, float c_fixed, const float* pts,
                      const float* normals, int64_t n, uint64_t seed, uint32_t walk_index, float* out_nu,
                      float* out_pdf, void* stream);
void wost_guide_free(wost_guide* g);

/* ------------------------------------------------------------ training
 * Online learning of the guide (Sec. 5.2 "Online Training Scheme").  The
 * per-record loss is
 *     l = -w [ log p_g(nu | Theta(x)) + e log( c sg(p_g) + (1 - c) p_u ) ],
 *     w = p_t / p_sample,
 * whose gradient w.r.t. Theta is the one-sample KL gradient of Sec. 4.2
 * (equation "one_sample_kld", with p_g the reflected mixture on Neumann
 * points, Sec. 4.3, or the plain mixture if the guide's reflection setting is
 * off) and w.r.t. c the selection-probability gradient of
 * Sec. 4.4 (equation "one_sample_sp"); sg is stop-gradient.  Records are
 * rows [begin, begin + count) of a wost_records buffer. */
typedef struct {
    float lr;               /* learning rate                                 */
    float beta1, beta2;     /* Adam moment decay rates                       */
    float eps;              /* Adam epsilon                                  */
    float e_mis;            /* fixed fraction e of the selection loss (0.2)  */
} wost_adam;

/* Fill the p_t field of every written record: p_t = |U - prefix| / T_next,
 * the walk's tail estimate of u at the next location (the reverse recursion
 * V_{k+1} of the walk's estimate), where U = walk_value[slot] is the final
 * estimate of the walk the record belongs to.  walk_value: device [n_slots],
 * the per-walk output of the wost_solve call that wrote the records. */
int wost_tail_pass(int32_t dim, const wost_records* rec, const float* walk_value, int64_t n_slots,
                   void* stream);
/* The training set of a batch (Sec. 5.2 "Online Training Scheme": the
 * guide is trained on the samples of the batch just taken): m rows drawn
 * uniformly with replacement from the rows `src` holds (its device count,
 * at most its capacity), by Philox4x32-10 under `seed`, copied into rows
 * 0..m-1 of `dst`; dst's count is set to m (0 if src is empty).  Minibatches
 * taken as contiguous ranges of dst then mix records of all the batch's
 * walks.  WOST_ESIZE if m exceeds dst's capacity. */
int wost_records_sample(int32_t dim, const wost_records* src, uint64_t seed, int64_t m, const wost_records* dst,
                        void* stream);
/* Workspace bytes for wost_guide_loss_bwd / wost_guide_train_step on `count`
 * records (per-workgroup partial weight gradients). */
int64_t wost_guide_train_workspace_bytes(const wost_guide* g, int64_t count);
/* Per-record loss l_i (device float [count]) with the current parameters
 * (fp16 shadow). */
int wost_guide_loss_fwd(const wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                        float e_mis, float* loss_out, void* stream);
/* grad += d/dparams sum_i scale * dloss_i * l_i (dloss device [count] or NULL
 * for all ones).  grad: device float [P] or NULL for the bound gradient.
 * Hash-grid activations are recomputed, not stored. */
int wost_guide_loss_bwd(const wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                        float e_mis, float scale, const float* dloss, float* grad, void* workspace,
                        int64_t ws_bytes, void* stream);
/* One Adam step (Kingma & Ba) on the master parameters with the bound
 * gradient, which is then zeroed; refreshes the fp16 shadow. */
int wost_guide_adam_step(wost_guide* g, const wost_adam* opt, void* stream);
/* One training step on records [begin, begin + count): mean loss (written to
 * device float *loss_out if not NULL), gradient, Adam, shadow refresh. */
int wost_guide_train_step(wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                          const wost_adam* opt, float* loss_out, void* workspace, int64_t ws_bytes,
                          void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * training step as wost_guide_train_step, with its workspace taken from a
 * library-owned device array of WOST_NOALLOC_SCRATCH_BYTES instead of a
 * caller buffer.  The call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); each device holds its own copy of the array
 * from library load until the process ends.  Every call on one device uses
 * that device's copy, so calls that overlap on a device (other streams, other
 * threads) race and must be ordered by the caller.  WOST_ESIZE if `count`
 * records need more workspace than the array holds
 * (wost_guide_train_workspace_bytes(g, count) > WOST_NOALLOC_SCRATCH_BYTES;
 * 2^18 records fit for the 2D and 3D guides of the benchmark scenes).  Other
 * arguments and errors as wost_guide_train_step. */
#define WOST_NOALLOC_SCRATCH_BYTES (128ll << 20)
int wost_guide_train_step_noalloc(wost_guide* g, const wost_records* rec, int64_t begin, int64_t count,
                                  const wost_adam* opt, float* loss_out, void* stream);

/* ------------------------------------------------------------ GPU hierarchy build
 * Linear BVH built on the GPU (Karras 2012; the paper's query library uses a
 * linear BVH, Sec. 5.3) over a primitive set for closest-point queries, in
 * the same four-wide node layout as the Dirichlet hierarchy that
 * wost_build_bvh writes.  Primitives are device float4 records: a 2D
 * segment (ax, ay, bx, by) per float4, a 3D triangle (a, b, c) packed in
 * three float4 (ax ay az bx | by bz cx cy | cz - - -).
 *
 * wost_lbvh_sizes: bytes of the node buffer (at most n - 1 four-wide nodes),
 * of the sorted primitive buffer and of the build workspace, for n >= 1
 * primitives (n below 2^25 - 64); WOST_EINVAL otherwise. */
int wost_lbvh_sizes(int32_t dim, int64_t n, int64_t* node_bytes, int64_t* prim_bytes, int64_t* ws_bytes);
/* Builds the hierarchy: Morton codes of the primitive centroids, radix sort,
 * binary radix tree, node boxes bottom-up, then four-wide nodes level by
 * level; a subtree of at most leaf_size (1..64) primitives becomes a leaf.
 * Outputs (caller-owned device buffers): nodes [node_bytes], prims_sorted
 * [prim_bytes] (the primitives in leaf order), orig int32 [n] (caller index
 * of each sorted primitive); host outputs *n_nodes and *levels (four-wide
 * depth).  workspace: device, 256-byte aligned, >= ws_bytes; prims, nodes and
 * prims_sorted 16-byte aligned.  Waits on `stream` (the level-by-level
 * collapse reads each level's size back). */
int wost_lbvh_build(int32_t dim, const float* prims, int64_t n, int32_t leaf_size, float* nodes,
                    float* prims_sorted, int32_t* orig, int32_t* n_nodes, int32_t* levels, void* workspace,
                    int64_t ws_bytes, void* stream);
/* Closest primitive to each of m points (device [m][dim]) in a hierarchy
 * from wost_lbvh_build: dist device float [m] (Euclidean distance), prim
 * device int32 [m] (caller index, -1 if none).  The traversal is the walk's
 * closest-Dirichlet-point query; its stack takes 3 (levels - 1) + 1 LDS
 * entries per lane (WOST_EUNSUPPORTED beyond 64 KB per workgroup). */
int wost_lbvh_closest(int32_t dim, const float* nodes, int32_t n_nodes, const float* prims_sorted,
                      const int32_t* orig, int32_t n_prims, int32_t levels, const float* pts, int64_t m,
                      float* dist, int32_t* prim, void* stream);
/* Uses a hierarchy from wost_lbvh_build over the geometry's Dirichlet
 * primitives (the same set, possibly moved) in place of the Dirichlet
 * section of the uploaded image, for wost_solve, wost_solve_wavefront and
 * wost_query; nodes NULL switches back to the image's own.  The buffers stay
 * caller-owned and must outlive their use.  n_prims must equal the
 * geometry's Dirichlet primitive count (else WOST_EINVAL), and the hierarchy
 * at most 14 levels deep (the traversal stack of wost_query, else
 * WOST_EUNSUPPORTED).  Host only. */
int wost_geom_use_dirichlet_lbvh(wost_geom* g, const float* nodes, int32_t n_nodes, const float* prims_sorted,
                                 const int32_t* orig, int32_t n_prims, int32_t levels);

/* ------------------------------------------------------------ launch tuning
 * Persistent walk workgroups (one wave each) per compute unit, 1..64, or 0
 * (the default) for as many as the launched kernel variant can keep resident
 * given its registers and LDS.  Process wide; affects throughput only, never
 * results. */
int wost_set_launch(int32_t waves_per_cu);
/* Walk pool of the persistent kernel.  Each wave keeps `slots_per_wave`
 * walks in flight (a multiple of 64 in [64, 8192]; 0 = the default of the
 * solve's dimension: 384 in 2D, 1536 in 3D) and advances all of them one
 * star per round, query by query; a lane whose query has finished takes the
 * next walk of that query's list, once at least `refill_batch` lanes (1..64;
 * 0 = default: 32 in 2D, 8 in 3D) are waiting or no lane is
 * still traversing.  Larger pools keep more lanes busy at the cost of
 * workspace.  Process wide; affects throughput and workspace size only,
 * never results.  Call wost_solve_workspace_bytes after changing it. */
int wost_set_walk_pool(int32_t slots_per_wave, int32_t refill_batch);
/* Traversal-cost instrumentation (process wide).  With a non-NULL device
 * uint64 [18] array, subsequent wost_solve calls run an instrumented kernel
 * variant that accumulates, per query type q (0 closest Dirichlet point,
 * 1 closest silhouette, 2 Neumann sample, 3 Neumann visibility, 4 source
 * visibility, 5 first hit): [2q] hierarchy nodes fetched and [2q+1]
 * primitives tested, summed over lanes; [12+q] wave-level loop iterations,
 * the sum over wave steps of the largest per-lane node count (a wave runs a
 * traversal for as long as its slowest lane).  NULL switches it off.
 * Results are unchanged; only throughput differs. */
int wost_set_cost_counters(uint64_t* dev_counters18);

#ifdef __cplusplus
}
#endif
#endif /* WOST_H */
