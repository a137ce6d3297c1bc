/*
 * FP64 walk-on-stars oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, brute-force CPU implementation of the walk-on-stars (WoSt)
 * estimator for the mixed Poisson problem (Laplacian u = f on the domain,
 * u = g on the Dirichlet part, du/dn = h on the Neumann part; paper Sec. 3.1,
 * the "linear_elliptic" equation), written for checking the GPU path.  Only
 * the tests, the package smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code with the GPU library.
 *
 * Every geometric query is exhaustive over all primitives; directions are
 * drawn uniformly (the original WoSt sampler, Sec. 4.1 "uniform directional
 * sampling").  Random numbers come from Philox4x32-10 (Salmon et al., SC'11),
 * implemented here from its published definition; the draw layout per step is
 * a fixed part of the interface so the GPU path can consume the identical
 * stream:
 *   counter = (point index, walk index of that point, step k, block b)
 *   key     = (seed low 32 bits, seed high 32 bits)
 *   b = 0 : direction words          b = 1 : Neumann (select, point, point), roulette
 *   b = 2 : source radius x3, source direction 0
 *   b = 3 : source direction 1, 3D vMF eta, 3D vMF phi, unused
 *   b = 4+i : 2D von Mises rejection iteration i
 * A 32-bit word w maps to the uniform (w >> 8) * 2^-24 in [0, 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ Philox */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    memcpy(out, c, sizeof(c));
}

static double u01(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }
/* (0, 1] variant for logarithms */

typedef struct {
    uint32_t key[2];
    uint32_t p, j;
} or_rng;

static void draw(const or_rng* g, uint32_t step, uint32_t block, double u[4])
{
    uint32_t ctr[4] = {g->p, g->j, step, block}, out[4];
    or_philox4x32_10(ctr, g->key, out);
    for (int i = 0; i < 4; ++i) u[i] = u01(out[i]);
}

/* ------------------------------------------------------------------ fields */

enum { F_ZERO = 0, F_CONST = 1, F_EXP_SIN = 2, F_RE_Z3 = 3, F_X2_MINUS_Y2 = 4, F_R2 = 5, F_GAUSS = 6 };

typedef struct {
    int kind;
    int n;               /* rows of params (gauss) or count */
    const double* params;
} or_field;

static double field_value(const or_field* f, int dim, const double* x)
{
    switch (f->kind) {
    case F_ZERO: return 0.0;
    case F_CONST: return f->params[0];
    case F_EXP_SIN: return exp(x[0]) * sin(x[1]);
    case F_RE_Z3: return x[0] * x[0] * x[0] - 3.0 * x[0] * x[1] * x[1];
    case F_X2_MINUS_Y2: return x[0] * x[0] - x[1] * x[1];
    case F_R2: { double s = 0; for (int i = 0; i < dim; ++i) s += x[i] * x[i]; return s; }
    case F_GAUSS: {
        double s = 0;
        for (int j = 0; j < f->n; ++j) {
            const double* row = f->params + j * (2 + dim);
            double d2 = 0;
            for (int i = 0; i < dim; ++i) { double t = x[i] - row[2 + i]; d2 += t * t; }
            s += row[0] * exp(-d2 / (2.0 * row[1] * row[1]));
        }
        return s;
    }
    }
    return NAN;
}

static void field_grad(const or_field* f, int dim, const double* x, double* gr)
{
    for (int i = 0; i < dim; ++i) gr[i] = 0.0;
    switch (f->kind) {
    case F_EXP_SIN: gr[0] = exp(x[0]) * sin(x[1]); gr[1] = exp(x[0]) * cos(x[1]); break;
    case F_RE_Z3: gr[0] = 3.0 * (x[0] * x[0] - x[1] * x[1]); gr[1] = -6.0 * x[0] * x[1]; break;
    case F_X2_MINUS_Y2: gr[0] = 2.0 * x[0]; gr[1] = -2.0 * x[1]; break;
    case F_R2: for (int i = 0; i < dim; ++i) gr[i] = 2.0 * x[i]; break;
    default: break;
    }
}

/* Neumann data: outward normal derivative h = du/dn_out at z on a primitive with
 * outward unit normal n_out.  A constant kind is the flux itself; a potential
 * kind phi gives h = grad(phi) . n_out. */
static double neumann_value(const or_field* h, int dim, const double* z, const double* n_out)
{
    if (h->kind == F_CONST) return h->params[0];
    double gr[3];
    field_grad(h, dim, z, gr);
    double s = 0;
    for (int i = 0; i < dim; ++i) s += gr[i] * n_out[i];
    return s;
}

/* ------------------------------------------------------------------ scene */

typedef struct {
    int dim;
    int64_t n_prims;
    double* pv;        /* [n_prims][dim][dim] vertex coordinates */
    double* n_out;     /* [n_prims][dim] outward unit normal */
    double* meas;      /* [n_prims] length / area */
    uint8_t* bc;       /* [n_prims] */
    /* silhouette candidates: 2D Neumann vertices, 3D Neumann edges */
    int64_t n_sil;
    double* sil_p;     /* [n_sil][2][dim] (2D: both rows = the vertex) */
    int32_t* sil_adj;  /* [n_sil][2] adjacent Neumann prims, -1 if none */
    double L;          /* AABB diagonal */
    double tau;        /* facing / self-hit tolerance, 1e-12 L */
} or_scene;

static double dot(int d, const double* a, const double* b)
{
    double s = 0; for (int i = 0; i < d; ++i) s += a[i] * b[i]; return s;
}

typedef struct { int64_t a, b, prim; } edge_rec;

static int edge_cmp(const void* x, const void* y)
{
    const edge_rec* p = (const edge_rec*)x; const edge_rec* q = (const edge_rec*)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return p->prim < q->prim ? -1 : (p->prim > q->prim);
}

or_scene* or_scene_create(int dim, const double* verts, int64_t n_verts,
                          const int32_t* prims, int64_t n_prims, const uint8_t* bc)
{
    if (dim != 2 && dim != 3) return NULL;
    or_scene* s = (or_scene*)calloc(1, sizeof(or_scene));
    s->dim = dim; s->n_prims = n_prims;
    s->pv = (double*)malloc(sizeof(double) * n_prims * dim * dim);
    s->n_out = (double*)malloc(sizeof(double) * n_prims * dim);
    s->meas = (double*)malloc(sizeof(double) * n_prims);
    s->bc = (uint8_t*)malloc(n_prims);
    memcpy(s->bc, bc, n_prims);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = 0; v < n_verts; ++v)
        for (int i = 0; i < dim; ++i) {
            double c = verts[v * dim + i];
            if (c < lo[i]) lo[i] = c;
            if (c > hi[i]) hi[i] = c;
        }
    double L2 = 0; for (int i = 0; i < dim; ++i) L2 += (hi[i] - lo[i]) * (hi[i] - lo[i]);
    s->L = sqrt(L2); s->tau = 1e-12 * s->L;
    for (int64_t q = 0; q < n_prims; ++q) {
        double* P = s->pv + q * dim * dim;
        for (int k = 0; k < dim; ++k)
            for (int i = 0; i < dim; ++i) P[k * dim + i] = verts[(int64_t)prims[q * dim + k] * dim + i];
        double* n = s->n_out + q * dim;
        if (dim == 2) {
            /* domain on the left of a->b: outward normal is the right normal */
            double ex = P[2] - P[0], ey = P[3] - P[1];
            double len = sqrt(ex * ex + ey * ey);
            n[0] = ey / len; n[1] = -ex / len; s->meas[q] = len;
        } else {
            double e1[3], e2[3], c[3];
            for (int i = 0; i < 3; ++i) { e1[i] = P[3 + i] - P[i]; e2[i] = P[6 + i] - P[i]; }
            c[0] = e1[1] * e2[2] - e1[2] * e2[1];
            c[1] = e1[2] * e2[0] - e1[0] * e2[2];
            c[2] = e1[0] * e2[1] - e1[1] * e2[0];
            double len = sqrt(dot(3, c, c));
            for (int i = 0; i < 3; ++i) n[i] = c[i] / len;
            s->meas[q] = 0.5 * len;
        }
    }
    /* silhouette candidates: every (vertex in 2D / edge in 3D) of a Neumann
       primitive, with its (up to two) adjacent Neumann primitives */
    int64_t n_rec = 0;
    int per = (dim == 2) ? 2 : 3;
    edge_rec* rec = (edge_rec*)malloc(sizeof(edge_rec) * (n_prims * per + 1));
    for (int64_t q = 0; q < n_prims; ++q) {
        if (!bc[q]) continue;
        if (dim == 2) {
            for (int k = 0; k < 2; ++k) { rec[n_rec].a = prims[q * 2 + k]; rec[n_rec].b = -1; rec[n_rec].prim = q; ++n_rec; }
        } else {
            for (int k = 0; k < 3; ++k) {
                int64_t a = prims[q * 3 + k], b = prims[q * 3 + (k + 1) % 3];
                rec[n_rec].a = a < b ? a : b; rec[n_rec].b = a < b ? b : a; rec[n_rec].prim = q; ++n_rec;
            }
        }
    }
    qsort(rec, n_rec, sizeof(edge_rec), edge_cmp);
    s->sil_p = (double*)malloc(sizeof(double) * (n_rec + 1) * 2 * dim);
    s->sil_adj = (int32_t*)malloc(sizeof(int32_t) * (n_rec + 1) * 2);
    int64_t ns = 0;
    for (int64_t i = 0; i < n_rec;) {
        int64_t j = i;
        while (j < n_rec && rec[j].a == rec[i].a && rec[j].b == rec[i].b) ++j;
        /* j - i adjacent prims; manifold boundaries give 1 or 2 */
        double* P = s->sil_p + ns * 2 * dim;
        for (int c = 0; c < dim; ++c) {
            P[c] = verts[rec[i].a * dim + c];
            P[dim + c] = (dim == 2) ? verts[rec[i].a * dim + c] : verts[rec[i].b * dim + c];
        }
        s->sil_adj[ns * 2 + 0] = (int32_t)rec[i].prim;
        s->sil_adj[ns * 2 + 1] = (j - i >= 2) ? (int32_t)rec[i + 1].prim : -1;
        ++ns;
        i = j;
    }
    s->n_sil = ns;
    free(rec);
    return s;
}

void or_scene_free(or_scene* s)
{
    if (!s) return;
    free(s->pv); free(s->n_out); free(s->meas); free(s->bc); free(s->sil_p); free(s->sil_adj);
    free(s);
}

int64_t or_scene_n_silhouette_candidates(const or_scene* s) { return s->n_sil; }

/* ------------------------------------------------------------------ geometry */

/* closest point on segment [a,b] to x */
static double closest_on_segment(int d, const double* x, const double* a, const double* b, double* out)
{
    double e[3], w[3];
    for (int i = 0; i < d; ++i) { e[i] = b[i] - a[i]; w[i] = x[i] - a[i]; }
    double ee = dot(d, e, e);
    double t = ee > 0 ? dot(d, w, e) / ee : 0.0;
    if (t < 0) t = 0; if (t > 1) t = 1;
    double d2 = 0;
    for (int i = 0; i < d; ++i) { out[i] = a[i] + t * e[i]; double u = x[i] - out[i]; d2 += u * u; }
    return sqrt(d2);
}

/* closest point on triangle: projection if it lies inside, else best of the
   three edges */
static double closest_on_triangle(const double* x, const double* P, double* out)
{
    const double *a = P, *b = P + 3, *c = P + 6;
    double e1[3], e2[3], w[3];
    for (int i = 0; i < 3; ++i) { e1[i] = b[i] - a[i]; e2[i] = c[i] - a[i]; w[i] = x[i] - a[i]; }
    double d11 = dot(3, e1, e1), d12 = dot(3, e1, e2), d22 = dot(3, e2, e2);
    double w1 = dot(3, w, e1), w2 = dot(3, w, e2);
    double det = d11 * d22 - d12 * d12;
    if (det > 0) {
        double u = (d22 * w1 - d12 * w2) / det;
        double v = (d11 * w2 - d12 * w1) / det;
        if (u >= 0 && v >= 0 && u + v <= 1) {
            double d2 = 0;
            for (int i = 0; i < 3; ++i) { out[i] = a[i] + u * e1[i] + v * e2[i]; double t = x[i] - out[i]; d2 += t * t; }
            return sqrt(d2);
        }
    }
    double best = INFINITY, tmp[3];
    const double* E[3][2] = {{a, b}, {b, c}, {c, a}};
    for (int k = 0; k < 3; ++k) {
        double dd = closest_on_segment(3, x, E[k][0], E[k][1], tmp);
        if (dd < best) { best = dd; memcpy(out, tmp, sizeof(tmp)); }
    }
    return best;
}

static double closest_on_prim(const or_scene* s, int64_t q, const double* x, double* out)
{
    const double* P = s->pv + q * s->dim * s->dim;
    if (s->dim == 2) return closest_on_segment(2, x, P, P + 2, out);
    return closest_on_triangle(x, P, out);
}

/* distance and closest point to the Dirichlet boundary (exhaustive) */
double or_closest_dirichlet_one(const or_scene* s, const double* x, double* xbar, int64_t* prim)
{
    double best = INFINITY, tmp[3];
    int64_t bq = -1;
    for (int64_t q = 0; q < s->n_prims; ++q) {
        if (s->bc[q]) continue;
        double d = closest_on_prim(s, q, x, tmp);
        if (d < best) { best = d; bq = q; memcpy(xbar, tmp, sizeof(double) * s->dim); }
    }
    if (prim) *prim = bq;
    return best;
}

/* primitive q faces x from the front if x lies on its domain side (ties count
   as front, so a walker sitting on q sees q as front) */
static int is_front(const or_scene* s, int64_t q, const double* x)
{
    const int d = s->dim;
    const double* a = s->pv + q * d * d;
    double w[3];
    for (int i = 0; i < d; ++i) w[i] = x[i] - a[i];
    /* inward normal = -n_out */
    return -dot(d, w, s->n_out + q * d) >= -s->tau;
}

/* distance to the nearest Neumann silhouette point seen from x (exhaustive),
   Sec. 3.2: a candidate is a silhouette when its adjacent Neumann primitives
   face x differently.  `own` (or -1) is a primitive x is known to lie on: it
   faces x from the front whatever the rounding of x (the walker's own
   primitive, as for a walker standing on the boundary) */
double or_silhouette_one(const or_scene* s, const double* x, int64_t own)
{
    double best = INFINITY, tmp[3];
    const int d = s->dim;
    for (int64_t k = 0; k < s->n_sil; ++k) {
        int32_t q0 = s->sil_adj[2 * k], q1 = s->sil_adj[2 * k + 1];
        int sil = (q1 < 0) ? 1 : ((q0 == own || is_front(s, q0, x)) != (q1 == own || is_front(s, q1, x)));
        if (!sil) continue;
        const double* P = s->sil_p + k * 2 * d;
        double dd = (d == 2) ? sqrt((x[0] - P[0]) * (x[0] - P[0]) + (x[1] - P[1]) * (x[1] - P[1]))
                             : closest_on_segment(3, x, P, P + 3, tmp);
        if (dd < best) best = dd;
    }
    return best;
}

/* ray x + t nu against primitive q; returns t or INFINITY */
static double ray_prim(const or_scene* s, int64_t q, const double* x, const double* nu)
{
    const double* P = s->pv + q * s->dim * s->dim;
    if (s->dim == 2) {
        double ex = P[2] - P[0], ey = P[3] - P[1];
        double den = nu[0] * ey - nu[1] * ex;
        if (den == 0.0) return INFINITY;
        double wx = P[0] - x[0], wy = P[1] - x[1];
        double t = (wx * ey - wy * ex) / den;
        double u = (wx * nu[1] - wy * nu[0]) / den;
        if (u < 0.0 || u > 1.0) return INFINITY;
        return t;
    }
    double e1[3], e2[3], pv[3], tv[3], qv[3];
    for (int i = 0; i < 3; ++i) { e1[i] = P[3 + i] - P[i]; e2[i] = P[6 + i] - P[i]; tv[i] = x[i] - P[i]; }
    pv[0] = nu[1] * e2[2] - nu[2] * e2[1];
    pv[1] = nu[2] * e2[0] - nu[0] * e2[2];
    pv[2] = nu[0] * e2[1] - nu[1] * e2[0];
    double det = dot(3, e1, pv);
    if (det == 0.0) return INFINITY;
    double u = dot(3, tv, pv) / det;
    if (u < 0.0 || u > 1.0) return INFINITY;
    qv[0] = tv[1] * e1[2] - tv[2] * e1[1];
    qv[1] = tv[2] * e1[0] - tv[0] * e1[2];
    qv[2] = tv[0] * e1[1] - tv[1] * e1[0];
    double v = dot(3, nu, qv) / det;
    if (v < 0.0 || u + v > 1.0) return INFINITY;
    return dot(3, e2, qv) / det;
}

/* first Neumann hit with t in (tau, tmax), skipping primitive `skip` */
double or_ray_neumann_one(const or_scene* s, const double* x, const double* nu, double tmax,
                          int64_t skip, int64_t* hit_prim)
{
    double best = tmax;
    int64_t bq = -1;
    for (int64_t q = 0; q < s->n_prims; ++q) {
        if (!s->bc[q] || q == skip) continue;
        double t = ray_prim(s, q, x, nu);
        if (t > s->tau && t < best) { best = t; bq = q; }
    }
    if (hit_prim) *hit_prim = bq;
    return bq >= 0 ? best : INFINITY;
}

/* no Neumann primitive (other than `skip` and `skip2`) crosses the open
   segment (x, z).  A point z on a primitive is tested with that primitive
   skipped: a flat primitive meets the segment to one of its points only at
   that point, so it can never block it. */
static int visible(const or_scene* s, const double* x, const double* z, int64_t skip, int64_t skip2)
{
    const int d = s->dim;
    double nu[3], len = 0;
    for (int i = 0; i < d; ++i) { nu[i] = z[i] - x[i]; len += nu[i] * nu[i]; }
    len = sqrt(len);
    if (len == 0) return 1;
    for (int i = 0; i < d; ++i) nu[i] /= len;
    for (int64_t q = 0; q < s->n_prims; ++q) {
        if (!s->bc[q] || q == skip || q == skip2) continue;
        double t = ray_prim(s, q, x, nu);
        if (t > s->tau && t < len - s->tau) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ kernels */


/* Green's function of the ball of radius r (zero Dirichlet on its sphere),
   -Laplacian G = delta, at distance rho from the centre */
static double green_ball(int d, double r, double rho)
{
    if (d == 2) return log(r / rho) / (2.0 * OR_PI);
    return (1.0 / rho - 1.0 / r) / (4.0 * OR_PI);
}

static void uniform_direction(int d, double u0, double u1, double* nu)
{
    if (d == 2) {
        double th = 2.0 * OR_PI * u0;
        nu[0] = cos(th); nu[1] = sin(th);
    } else {
        double z = 1.0 - 2.0 * u0, ph = 2.0 * OR_PI * u1;
        double rr = sqrt(fmax(0.0, 1.0 - z * z));
        nu[0] = rr * cos(ph); nu[1] = rr * sin(ph); nu[2] = z;
    }
}

/* ------------------------------------------------------------------ walk */

typedef struct {
    or_field g, h, f;
    double eps, r_min;
    int32_t max_steps, rr_start;
    double rr_q;
} or_problem;

typedef struct {
    double value;
    int32_t steps;        /* stars visited: distance queries, terminating one included */
    int32_t status;       /* 0 reached eps-shell, 1 step cap, 2 roulette kill */
    double terminal;      /* g(xbar) at termination (0 if killed) */
    double t_final;       /* throughput at termination */
} or_walk_result;

/* Optional per-step trace (for the reverse-recursion check): c_k and w_k. */
typedef struct {
    double* c;   /* [cap] contribution N_k + S_k of step k */
    double* w;   /* [cap] weight of the recursive term at step k (roulette folded in) */
    int32_t cap;
    int32_t n;
} or_trace;

static or_walk_result walk_one(const or_scene* s, const or_problem* pb, const double* x0,
                               const or_rng* g, or_trace* tr)
{
    const int d = s->dim;
    double x[3] = {0, 0, 0}, n_in[3] = {0, 0, 0}, xbar[3];
    for (int i = 0; i < d; ++i) x[i] = x0[i];
    int onN = 0;
    int64_t on_prim = -1;
    double T = 1.0, U = 0.0;
    or_walk_result res = {0};
    const int has_h = pb->h.kind != F_ZERO;
    const int has_f = pb->f.kind != F_ZERO;
    for (int32_t k = 0;; ++k) {
        double u[4];
        if (k >= pb->rr_start && k > 0) {
            draw(g, (uint32_t)k, 1, u);
            if (u[3] >= pb->rr_q) { res.status = 2; res.terminal = 0.0; break; }
            T /= pb->rr_q;
            if (tr && tr->n > 0) tr->w[tr->n - 1] /= pb->rr_q;
        }
        res.steps = k + 1;
        double dD = or_closest_dirichlet_one(s, x, xbar, NULL);
        if (dD <= pb->eps || k >= pb->max_steps) {
            double gv = field_value(&pb->g, d, xbar);
            U += T * gv;
            res.terminal = gv;
            res.status = (dD <= pb->eps) ? 0 : 1;
            break;
        }
        double dS = or_silhouette_one(s, x, -1);
        double r = fmin(dD, dS);
        if (r < pb->r_min) r = pb->r_min;
        const double alpha = onN ? 0.5 : 1.0;
        double contrib = 0.0;

        /* Neumann contribution: z uniform over the Neumann primitives that
           overlap the ball (pdf 1/A), kept if it lies in the star */
        if (has_h) {
            draw(g, (uint32_t)k, 1, u);
            double A = 0.0, tmp[3];
            for (int64_t q = 0; q < s->n_prims; ++q)
                if (s->bc[q] && closest_on_prim(s, q, x, tmp) < r) A += s->meas[q];
            if (A > 0.0) {
                double target = u[0] * A, acc = 0.0;
                int64_t sel = -1;
                for (int64_t q = 0; q < s->n_prims; ++q) {
                    if (!(s->bc[q] && closest_on_prim(s, q, x, tmp) < r)) continue;
                    sel = q;
                    acc += s->meas[q];
                    if (target < acc) break;
                }
                const double* P = s->pv + sel * d * d;
                double z[3];
                if (d == 2) {
                    for (int i = 0; i < 2; ++i) z[i] = P[i] + u[1] * (P[2 + i] - P[i]);
                } else {
                    double sq = sqrt(u[1]);
                    for (int i = 0; i < 3; ++i)
                        z[i] = P[i] * (1.0 - sq) + P[3 + i] * sq * (1.0 - u[2]) + P[6 + i] * sq * u[2];
                }
                double dz[3], rho = 0.0;
                for (int i = 0; i < d; ++i) { dz[i] = z[i] - x[i]; rho += dz[i] * dz[i]; }
                rho = sqrt(rho);
                int ok = rho < r && rho > 0.0;
                if (ok && onN && dot(d, dz, n_in) < -s->tau) ok = 0;
                if (ok && !visible(s, x, z, onN ? on_prim : -1, sel)) ok = 0;
                if (ok) {
                    double hv = neumann_value(&pb->h, d, z, s->n_out + sel * d);
                    contrib += green_ball(d, r, rho) * hv * A / alpha;
                }
            }
        }
        /* source contribution: y = x + s r nu' with s from the radial law of
           the ball's Green's function (density proportional to G rho^(d-1)) */
        if (has_f) {
            double ua[4], ub[4];
            draw(g, (uint32_t)k, 2, ua);
            draw(g, (uint32_t)k, 3, ub);
            double sr;
            if (d == 2) {
                sr = sqrt(ua[0] * ua[1]);
            } else {
                double a = ua[0], b = ua[1], c = ua[2];
                sr = fmax(fmin(a, b), fmin(fmax(a, b), c));   /* median */
            }
            double nu2[3], y[3];
            uniform_direction(d, ua[3], ub[0], nu2);
            for (int i = 0; i < d; ++i) y[i] = x[i] + sr * r * nu2[i];
            int ok = sr > 0.0;
            if (ok && onN && dot(d, nu2, n_in) <= 0.0) ok = 0;
            if (ok && !visible(s, x, y, onN ? on_prim : -1, -1)) ok = 0;
            if (ok) contrib += -(r * r / (2.0 * d)) * field_value(&pb->f, d, y) / alpha;
        }
        U += T * contrib;

        /* direction: uniform on the sphere, folded onto the valid hemisphere on
           a Neumann boundary; weight 1 / (|S| alpha p) = 1 */
        draw(g, (uint32_t)k, 0, u);
        double nu[3];
        uniform_direction(d, u[0], u[1], nu);
        if (onN) {
            double c = dot(d, nu, n_in);
            if (c < 0) for (int i = 0; i < d; ++i) nu[i] -= 2.0 * c * n_in[i];
        }
        const double w = 1.0;
        if (tr && tr->n < tr->cap) { tr->c[tr->n] = contrib; tr->w[tr->n] = w; tr->n++; }

        int64_t hp;
        double t = or_ray_neumann_one(s, x, nu, r, onN ? on_prim : -1, &hp);
        if (hp >= 0) {
            for (int i = 0; i < d; ++i) x[i] += t * nu[i];
            const double* no = s->n_out + hp * d;
            double c = dot(d, no, nu);
            /* normal on the walker's side: opposite to the arriving direction */
            for (int i = 0; i < d; ++i) n_in[i] = (c > 0) ? -no[i] : no[i];
            onN = 1; on_prim = hp;
        } else {
            for (int i = 0; i < d; ++i) x[i] += r * nu[i];
            onN = 0; on_prim = -1;
        }
        T *= w;
    }
    res.value = U;
    res.t_final = T;
    return res;
}

/*
 * Uniform-sampling WoSt over n_points query points x wpp walks.
 * Walk (p, j) uses the Philox stream keyed by `seed` with counter
 * (p, walk_offset + j, step, block).  Outputs are accumulated (+=) per point:
 * sum, sum of squares, count and total steps.  Optional per-walk arrays are
 * indexed p * wpp + j.  `point_ids` (optional) replaces p in the counter by
 * point_ids[p], so a sample of a larger point set reproduces that set's walks.
 * Returns 0 on success.
 */
int or_solve(const or_scene* s, const or_problem* pb, const double* pts, int64_t n_points,
             const int64_t* point_ids, int32_t wpp, uint64_t seed, uint64_t walk_offset,
             double* sum, double* sumsq, int64_t* count, int64_t* steps,
             double* walk_value, int32_t* walk_steps, int32_t* walk_status, int nthreads)
{
    if (!s || !pb || wpp <= 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_points; ++p) {
        double su = 0, sq = 0;
        int64_t st = 0;
        for (int32_t j = 0; j < wpp; ++j) {
            or_rng g;
            g.key[0] = (uint32_t)seed; g.key[1] = (uint32_t)(seed >> 32);
            g.p = (uint32_t)(point_ids ? point_ids[p] : p);
            g.j = (uint32_t)(walk_offset + (uint64_t)j);
            or_walk_result r = walk_one(s, pb, pts + p * s->dim, &g, NULL);
            su += r.value; sq += r.value * r.value; st += r.steps;
            if (walk_value) walk_value[p * wpp + j] = r.value;
            if (walk_steps) walk_steps[p * wpp + j] = r.steps;
            if (walk_status) walk_status[p * wpp + j] = r.status;
        }
        sum[p] += su; sumsq[p] += sq; count[p] += wpp;
        if (steps) steps[p] += st;
    }
    return 0;
}

/* One walk with its per-step (c_k, w_k) trace; returns the number of trace
   entries.  Used to check the reverse (tail) recursion against the forward sum. */
int32_t or_walk_trace(const or_scene* s, const or_problem* pb, const double* x0,
                      uint64_t seed, uint32_t p, uint32_t j, double* c, double* w, int32_t cap,
                      double* value, double* terminal, int32_t* status)
{
    or_rng g;
    g.key[0] = (uint32_t)seed; g.key[1] = (uint32_t)(seed >> 32);
    g.p = p; g.j = j;
    or_trace tr = {c, w, cap, 0};
    or_walk_result r = walk_one(s, pb, x0, &g, &tr);
    *value = r.value; *terminal = r.terminal; *status = r.status;
    return tr.n;
}

/* Step-0 contribution N_0 + S_0 (Neumann and source terms of the first star)
   of walks j = j0 .. j0 + n - 1 of point p started at x0; 0 where a walk ends
   at step 0.  Its mean over walks estimates the first star's Green's-function
   integrals of h and f (Sec. 3.2, equation "wost_estm"), which the tests
   compare with quadrature. */
int or_first_step(const or_scene* s, const or_problem* pb, const double* x0, uint64_t seed, uint32_t p,
                  uint32_t j0, int64_t n, double* c0)
{
    if (!s || !pb || n < 0) return -1;
    or_problem one = *pb;
    one.max_steps = 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        or_rng g;
        g.key[0] = (uint32_t)seed; g.key[1] = (uint32_t)(seed >> 32);
        g.p = p; g.j = j0 + (uint32_t)i;
        double c = 0.0, w = 0.0;
        or_trace tr = {&c, &w, 1, 0};
        walk_one(s, &one, x0, &g, &tr);
        c0[i] = tr.n ? c : 0.0;
    }
    return 0;
}

/* batch query helpers for parity tests */
void or_closest_dirichlet(const or_scene* s, const double* x, int64_t n, double* dist, double* xbar)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        dist[i] = or_closest_dirichlet_one(s, x + i * s->dim, xbar + i * s->dim, NULL);
}

/* on_prim: NULL, or per point the caller primitive it lies on (-1 = none) */
void or_silhouette(const or_scene* s, const double* x, int64_t n, const int64_t* on_prim, double* dist)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) dist[i] = or_silhouette_one(s, x + i * s->dim, on_prim ? on_prim[i] : -1);
}

void or_ray_neumann(const or_scene* s, const double* x, const double* nu, const double* tmax,
                    int64_t n, double* t, int64_t* prim)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        t[i] = or_ray_neumann_one(s, x + i * s->dim, nu + i * s->dim, tmax[i], -1, prim + i);
}

double or_green_ball(int d, double r, double rho) { return green_ball(d, r, rho); }

double or_field_value(int kind, int n, const double* params, int dim, const double* x)
{
    or_field f = {kind, n, params};
    return field_value(&f, dim, x);
}

/* Facing / self-intersection tolerance relative to the AABB diagonal (default
   1e-12).  Query-parity tests set the GPU path's FP32 tolerance here so that
   both sides take facing decisions with the same margin. */
void or_scene_set_tolerance(or_scene* s, double tau_rel) { s->tau = tau_rel * s->L; }

/* Batched Philox4x32-10: out[i] = philox(ctr[i], key) for i < n. */
void or_philox4x32_10_batch(const uint32_t* ctr, int64_t n, const uint32_t key[2], uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i) or_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}
