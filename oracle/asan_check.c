/*
 * Memory-error check of the FP64 oracle: built as one translation unit with
 * the oracle source under AddressSanitizer and UndefinedBehaviorSanitizer
 * (gcc -fsanitize=address,undefined), it drives every entry point on small
 * 2D and 3D scenes with mixed boundary conditions, a source term and walks
 * long enough for Russian roulette to act.  Test infrastructure, like the
 * oracle itself.  Exit status 0 and "asan oracle ok" on success.  Built with
 * WOST_PLANT_OVERRUN it hands the solver a per-walk buffer one entry short,
 * which the sanitizer must report.
 */
#include "wost_oracle.c"

#include <stdio.h>

static const double kPi = 3.14159265358979323846;

static int finite_all(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* unit circle of n segments, the upper half Neumann; u = Re z^3 */
static int check_2d(void)
{
    enum { N = 48, P = 16, WPP = 8 };
    double v[2 * N];
    int32_t pr[2 * N];
    uint8_t bc[N];
    for (int i = 0; i < N; ++i) {
        const double t = 2.0 * kPi * i / N;
        v[2 * i] = cos(t);
        v[2 * i + 1] = sin(t);
        pr[2 * i] = i;
        pr[2 * i + 1] = (i + 1) % N;
        bc[i] = sin(t + kPi / N) > 0.0;
    }
    or_scene* s = or_scene_create(2, v, N, pr, N, bc);
    if (!s) return 1;
    or_problem pb;
    memset(&pb, 0, sizeof(pb));
    pb.g.kind = F_RE_Z3;
    pb.h.kind = F_RE_Z3;
    pb.f.kind = F_ZERO;
    pb.eps = 1e-3;
    pb.max_steps = 4096;
    pb.rr_start = 4;
    pb.rr_q = 0.9;
    double pts[2 * P];
    for (int p = 0; p < P; ++p) {
        pts[2 * p] = 0.6 * cos(0.37 * p);
        pts[2 * p + 1] = 0.6 * sin(0.37 * p);
    }
    double sum[P] = {0}, sq[P] = {0}, wv[P * WPP];
    int64_t cnt[P] = {0}, steps[P] = {0};
    int32_t ws[P * WPP], st[P * WPP];
#ifdef WOST_PLANT_OVERRUN
    /* the sanitizer's own check: a per-walk buffer one walk too short */
    double* short_wv = (double*)malloc(sizeof(double) * (P * WPP - 1));
    (void)or_solve(s, &pb, pts, P, NULL, WPP, 2410, 0, sum, sq, cnt, steps, short_wv, ws, st, 1);
    free(short_wv);
#endif
    if (or_solve(s, &pb, pts, P, NULL, WPP, 2410, 0, sum, sq, cnt, steps, wv, ws, st, 1) != 0) return 2;
    if (!finite_all(sum, P) || !finite_all(wv, P * WPP)) return 3;
    double dist[P], xbar[2 * P], sil[P], t[P], tmax[P], nu[2 * P];
    int64_t own[P], hit[P];
    for (int p = 0; p < P; ++p) {
        own[p] = -1;
        tmax[p] = 3.0;
        nu[2 * p] = cos(1.1 * p);
        nu[2 * p + 1] = sin(1.1 * p);
    }
    or_closest_dirichlet(s, pts, P, dist, xbar);
    or_silhouette(s, pts, P, own, sil);
    or_ray_neumann(s, pts, nu, tmax, P, t, hit);
    double c[64], w[64], value = 0, terminal = 0;
    int32_t status = 0;
    (void)or_walk_trace(s, &pb, pts, 2410, 0, 0, c, w, 64, &value, &terminal, &status);
    or_scene_set_tolerance(s, 1e-9);
    or_scene_free(s);
    return finite_all(dist, P) && finite_all(xbar, 2 * P) ? 0 : 4;
}

/* axis-aligned cube of 12 triangles, the top and one side Neumann; u = x^2 - y^2
   with a Gaussian source */
static int check_3d(void)
{
    enum { P = 8, WPP = 4 };
    const double v[8 * 3] = {-1, -1, -1, 1, -1, -1, 1, 1, -1, -1, 1, -1, -1, -1, 1, 1, -1, 1, 1, 1, 1, -1, 1, 1};
    /* outward winding: (b - a) x (c - a) points out of the cube */
    const int32_t pr[12 * 3] = {0, 2, 1, 0, 3, 2, 4, 5, 6, 4, 6, 7, 0, 1, 5, 0, 5, 4,
                                2, 3, 7, 2, 7, 6, 1, 2, 6, 1, 6, 5, 0, 4, 7, 0, 7, 3};
    const uint8_t bc[12] = {0, 0, 1, 1, 0, 0, 0, 0, 1, 1, 0, 0};
    or_scene* s = or_scene_create(3, v, 8, pr, 12, bc);
    if (!s) return 11;
    const double gauss[5] = {1.5, 0.3, 0.1, -0.2, 0.3};
    or_problem pb;
    memset(&pb, 0, sizeof(pb));
    pb.g.kind = F_X2_MINUS_Y2;
    pb.h.kind = F_X2_MINUS_Y2;
    pb.f.kind = F_GAUSS;
    pb.f.n = 1;
    pb.f.params = gauss;
    pb.eps = 1e-3;
    pb.max_steps = 4096;
    pb.rr_start = 4;
    pb.rr_q = 0.9;
    double pts[3 * P];
    for (int p = 0; p < P; ++p) {
        pts[3 * p] = 0.5 * cos(0.7 * p);
        pts[3 * p + 1] = 0.5 * sin(0.7 * p);
        pts[3 * p + 2] = 0.1 * p - 0.35;
    }
    double sum[P] = {0}, sq[P] = {0}, wv[P * WPP];
    int64_t cnt[P] = {0}, steps[P] = {0};
    int32_t ws[P * WPP], st[P * WPP];
    if (or_solve(s, &pb, pts, P, NULL, WPP, 18944, 0, sum, sq, cnt, steps, wv, ws, st, 1) != 0) return 12;
    if (!finite_all(sum, P) || !finite_all(wv, P * WPP)) return 13;
    double dist[P], xbar[3 * P], sil[P];
    int64_t own[P];
    for (int p = 0; p < P; ++p) own[p] = -1;
    or_closest_dirichlet(s, pts, P, dist, xbar);
    or_silhouette(s, pts, P, own, sil);
    or_scene_free(s);
    return finite_all(dist, P) ? 0 : 14;
}

int main(void)
{
    const int r2 = check_2d();
    const int r3 = check_3d();
    if (r2 || r3) {
        printf("asan oracle check failed: %d %d\n", r2, r3);
        return 1;
    }
    printf("asan oracle ok\n");
    return 0;
}
