"""Pins of the FP64 walk-on-stars oracle against facts fixed by the paper and
by mathematics (closed forms, invariants, published test vectors, brute force).

None of these tests needs a GPU.  Each one is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign, a transposed operand, a
wrong normal orientation) makes it fail.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import scenes
from tests.stats import zscore_check

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- RNG

def test_philox_known_answers(oracle_lib):
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = oracle_lib.philox4x32_10(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


# ----------------------------------------------------------------------------- geometry

def _regular_polygon_scene(n=128, bc_value=0):
    s = scenes.scene_c1()
    s.bc[:] = bc_value
    return s


def test_closest_point_regular_polygon_closed_form(oracle_lib):
    s = _regular_polygon_scene()
    o = oracle_lib.OracleScene(s)
    # centre: distance is the apothem cos(pi/128)
    d, xb = o.closest_dirichlet(np.zeros((1, 2)))
    assert abs(d[0] - math.cos(math.pi / 128)) < 1e-14
    # points on rays through edge midpoints: distance apothem - rho
    k = np.arange(0, 128, 7)
    ang = 2 * np.pi * (k + 0.5) / 128
    rho = np.linspace(0.0, 0.9, k.size)
    x = np.stack([rho * np.cos(ang), rho * np.sin(ang)], 1)
    d, xb = o.closest_dirichlet(x)
    np.testing.assert_allclose(d, math.cos(math.pi / 128) - rho, atol=1e-13)
    # closest point lies on the edge midpoint ray
    np.testing.assert_allclose(np.hypot(xb[:, 0], xb[:, 1]), math.cos(math.pi / 128), atol=1e-13)


def test_closest_point_vs_dense_boundary_sampling(oracle_lib):
    s = scenes.scene_c2()
    o = oracle_lib.OracleScene(s)
    rng = np.random.default_rng(3)
    x = s.points[rng.choice(s.n_points, 64, replace=False)]
    d, xb = o.closest_dirichlet(x)
    # dense sampling of the Dirichlet segments: 64 samples per segment
    D = s.prims[s.bc == 0]
    a, b = s.verts[D[:, 0]], s.verts[D[:, 1]]
    t = (np.arange(64) + 0.5) / 64
    pts = (a[:, None, :] + t[None, :, None] * (b - a)[:, None, :]).reshape(-1, 2)
    seg = np.max(np.hypot(*(b - a).T))
    for i in range(x.shape[0]):
        dd = np.min(np.hypot(*(pts - x[i]).T))
        assert d[i] <= dd + 1e-12
        assert dd <= d[i] + seg / 64
    # the returned closest point is at the returned distance and on a segment
    np.testing.assert_allclose(np.hypot(*(xb - x).T), d, rtol=1e-12)


def _l_shape():
    """L-shaped domain [-1,1]^2 minus the quadrant x>0, y<0; all Neumann except
    the far-left edge.  Reflex vertex at the origin."""
    V = np.array([[-1, -1], [0, -1], [0, 0], [1, 0], [1, 1], [-1, 1]], float)
    P = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 5], [5, 0]], np.int32)
    bc = np.array([1, 1, 1, 1, 1, 0], np.uint8)
    return scenes.Scene("L", 2, V, P, bc, np.zeros((1, 2)), g=(0, np.zeros(0)), h=(0, np.zeros(0)),
                        f=(0, np.zeros(0)), u_exact=None)


def test_silhouette_l_shape_closed_form(oracle_lib):
    o = oracle_lib.OracleScene(_l_shape())
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.95, 0.95, size=(4000, 2))
    x = x[~((x[:, 0] > 0) & (x[:, 1] < 0))]
    dS = o.silhouette(x)
    # edge (0,-1)->(0,0) has inward normal -x: front iff x <= 0;
    # edge (0,0)->(1,0) has inward normal +y: front iff y >= 0.
    sil = (x[:, 0] <= 0) != (x[:, 1] >= 0)
    expect = np.where(sil, np.hypot(x[:, 0], x[:, 1]), np.inf)
    # the other Neumann vertices are convex (never silhouettes) except the
    # vertex (-1,-1) and (-1,1) which touch the Dirichlet edge: they have one
    # Neumann neighbour and always count
    ends = np.minimum(np.hypot(x[:, 0] + 1, x[:, 1] + 1), np.hypot(x[:, 0] + 1, x[:, 1] - 1))
    expect = np.minimum(expect, ends)
    np.testing.assert_allclose(dS, expect, rtol=1e-14)


def test_silhouette_convex_polygon_is_empty(oracle_lib):
    s = _regular_polygon_scene(bc_value=1)
    o = oracle_lib.OracleScene(s)
    dS = o.silhouette(s.points)
    assert np.all(np.isinf(dS))


def test_silhouette_from_the_boundary_of_a_convex_polygon(oracle_lib):
    """Seen from a point on a convex polygon's boundary no vertex is a
    silhouette.  Points rounded off their edge by ~1e-8 would see their own
    edge from behind, so the edge each point lies on is passed as its own
    primitive, which faces it from the front (a walker standing on it)."""
    s = _regular_polygon_scene(bc_value=1)
    o = oracle_lib.OracleScene(s)
    rng = np.random.default_rng(5)
    q = rng.integers(0, len(s.prims), 2000)
    a, b = s.verts[s.prims[q, 0]], s.verts[s.prims[q, 1]]
    t = rng.uniform(0.05, 0.95, (2000, 1))
    x = np.asarray(a + t * (b - a), np.float32).astype(np.float64)
    assert np.all(np.isinf(o.silhouette(x, on_prim=q)))
    # without it, the points that lie outside their edge's line see its two
    # ends as silhouettes (the rounding is what decides)
    # (facing tolerance 1e-12 of the AABB diagonal 2 sqrt 2, inward normal =
    # left normal of the counter-clockwise edges)
    e = b - a
    nin = np.stack([-e[:, 1], e[:, 0]], 1) / np.linalg.norm(e, axis=1, keepdims=True)
    sd = np.einsum("ij,ij->i", x - a, nin)
    tau = 1e-12 * 2.0 * math.sqrt(2.0)
    plain = o.silhouette(x)
    clear = np.abs(sd + tau) > 1e-15
    assert (sd < -tau).any()
    np.testing.assert_array_equal(np.isfinite(plain)[clear], (sd < -tau)[clear])


def test_star_radius_gives_star_shaped_region(oracle_lib):
    """Within r = min(d_D, d_S) every ray from x crosses the Neumann boundary
    at most once (the star region is star-shaped as seen from x)."""
    s = scenes.scene_c2()
    o = oracle_lib.OracleScene(s)
    rng = np.random.default_rng(7)
    # points near the outer boundary, where silhouettes matter
    r_pts = np.hypot(*s.points.T)
    cand = np.where(r_pts > 0.75)[0]
    x = s.points[rng.choice(cand, 24, replace=False)]
    dD, _ = o.closest_dirichlet(x)
    dS = o.silhouette(x)
    N = s.prims[s.bc == 1]
    a, b = s.verts[N[:, 0]], s.verts[N[:, 1]]
    th = np.linspace(0, 2 * np.pi, 1440, endpoint=False)
    nus = np.stack([np.cos(th), np.sin(th)], 1)
    n_checked = 0
    for i in range(x.shape[0]):
        r = min(dD[i], dS[i])
        e = b - a
        for nu in nus:
            den = nu[0] * e[:, 1] - nu[1] * e[:, 0]
            w = a - x[i]
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (w[:, 0] * e[:, 1] - w[:, 1] * e[:, 0]) / den
                u = (w[:, 0] * nu[1] - w[:, 1] * nu[0]) / den
            hits = (u >= 0) & (u <= 1) & (t > 1e-12) & (t < r * (1 - 1e-9))
            assert hits.sum() <= 1
            n_checked += 1
    assert n_checked > 0


def test_ray_axis_aligned_square_closed_form(oracle_lib):
    V = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], float)
    P = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.int32)
    sq = scenes.Scene("sq", 2, V, P, np.ones(4, np.uint8), np.zeros((1, 2)), g=(0, np.zeros(0)),
                      h=(0, np.zeros(0)), f=(0, np.zeros(0)), u_exact=None)
    o = oracle_lib.OracleScene(sq)
    rng = np.random.default_rng(2)
    x = rng.uniform(-0.9, 0.9, size=(500, 2))
    th = rng.uniform(0, 2 * np.pi, 500)
    nu = np.stack([np.cos(th), np.sin(th)], 1)
    t, prim = o.ray_neumann(x, nu, np.full(500, 10.0))
    with np.errstate(divide="ignore"):
        tx = np.where(nu[:, 0] > 0, (1 - x[:, 0]) / nu[:, 0], (-1 - x[:, 0]) / nu[:, 0])
        ty = np.where(nu[:, 1] > 0, (1 - x[:, 1]) / nu[:, 1], (-1 - x[:, 1]) / nu[:, 1])
    np.testing.assert_allclose(t, np.minimum(tx, ty), rtol=1e-12)
    # beyond tmax there is no hit
    t2, prim2 = o.ray_neumann(x, nu, np.minimum(tx, ty) * 0.5)
    assert np.all(prim2 < 0) and np.all(np.isinf(t2))


def test_closest_point_triangle_vs_dense_sampling(oracle_lib):
    s = scenes.scene_cube_box()
    o = oracle_lib.OracleScene(s)
    rng = np.random.default_rng(4)
    x = rng.uniform(-0.99, 0.99, size=(200, 3))
    d, xb = o.closest_dirichlet(x)
    expect = np.min(1.0 - np.abs(x), axis=1)
    np.testing.assert_allclose(d, expect, atol=1e-13)
    # points outside the cube: distance to the box
    y = rng.uniform(-2, 2, size=(200, 3))
    y = y[np.max(np.abs(y), 1) > 1.0]
    d, _ = o.closest_dirichlet(y)
    ex = np.linalg.norm(np.maximum(np.abs(y) - 1.0, 0.0), axis=1)
    np.testing.assert_allclose(d, ex, atol=1e-13)


# ----------------------------------------------------------------------------- Green's function

@pytest.mark.parametrize("d", [2, 3])
def test_green_ball_integral(oracle_lib, d):
    """Integral of the ball's Green's function over the ball is r^2 / (2d),
    and it vanishes on the sphere."""
    r = 0.37
    area = 2 * np.pi if d == 2 else 4 * np.pi
    val, _ = integrate.quad(lambda rho: oracle_lib.green_ball(d, r, rho) * area * rho ** (d - 1), 0, r,
                            limit=200)
    assert abs(val - r * r / (2 * d)) < 1e-9
    assert abs(oracle_lib.green_ball(d, r, r)) < 1e-15


@pytest.mark.parametrize("d", [2, 3])
def test_green_ball_fundamental_solution(oracle_lib, d):
    """-Laplacian G = 0 away from the centre (radial Laplacian by finite
    differences) and the flux through a small sphere is -1."""
    r, rho, h = 0.5, 0.2, 1e-4
    G = lambda q: oracle_lib.green_ball(d, r, q)  # noqa: E731
    lap = (G(rho + h) - 2 * G(rho) + G(rho - h)) / h ** 2 + (d - 1) / rho * (G(rho + h) - G(rho - h)) / (2 * h)
    assert abs(lap) < 1e-4
    dG = (G(rho + h) - G(rho - h)) / (2 * h)
    area = 2 * np.pi * rho if d == 2 else 4 * np.pi * rho ** 2
    assert abs(dG * area + 1.0) < 1e-6


# ----------------------------------------------------------------------------- estimator

def _exact(s, pts):
    from oracle import field_value
    return np.array([field_value(s.u_exact, s.dim, p) for p in pts])


def test_c1_laplace_matches_closed_form(oracle_lib):
    s = scenes.scene_c1()
    o = oracle_lib.OracleScene(s)
    r = o.solve(wpp=256)
    m, se, n = oracle_lib.estimates(r)
    zscore_check(m, se, _exact(s, s.points), n, label="C1")


def test_c1_poisson_pins_source_sign(oracle_lib):
    """Manufactured u = |x|^2 with Laplacian u = 4: fixes the sign of the source
    contribution (the estimator adds -(r^2/2d) f)."""
    s = scenes.scene_c1_poisson()
    o = oracle_lib.OracleScene(s)
    r = o.solve(wpp=256)
    m, se, n = oracle_lib.estimates(r)
    # epsilon-shell bias: terminal g(xbar) vs u(x) differ by <= eps |grad u| = 2e-3
    zscore_check(m, se, _exact(s, s.points), n, bias_slack=0.6, label="C1-poisson")
    # a flipped source sign would be off by 2 (1 - |x|^2) on average
    assert np.mean(np.abs(m - _exact(s, s.points))) < 0.05


def test_half_neumann_disk_pins_neumann_sign(oracle_lib):
    """Upper arc Neumann with h = d(Re z^3)/dn_out, lower arc Dirichlet."""
    s = scenes.scene_halfdisk_neumann()
    o = oracle_lib.OracleScene(s)
    r = o.solve(wpp=1024)
    m, se, n = oracle_lib.estimates(r)
    zscore_check(m, se, _exact(s, s.points), n, label="halfdisk")


def test_c2_subset_matches_re_z3(oracle_lib):
    s = scenes.scene_c2()
    idx = np.arange(0, s.n_points, 97)[:256]
    o = oracle_lib.OracleScene(s)
    r = o.solve(points=s.points[idx], wpp=128)
    m, se, n = oracle_lib.estimates(r)
    zscore_check(m, se, _exact(s, s.points[idx]), n, label="C2 subset")


def test_cube_3d_laplace(oracle_lib):
    s = scenes.scene_cube_box()
    o = oracle_lib.OracleScene(s)
    r = o.solve(wpp=256)
    m, se, n = oracle_lib.estimates(r)
    zscore_check(m, se, _exact(s, s.points), n, label="cube")


def test_walk_streams_are_reproducible_and_batch_invariant(oracle_lib):
    """Walk (p, j) depends only on (seed, p, j): two calls covering walks
    [0, 8) and [8, 16) reproduce one call over [0, 16)."""
    s = scenes.scene_c1()
    o = oracle_lib.OracleScene(s)
    pts = s.points[:16]
    a = o.solve(points=pts, wpp=16, per_walk=True)
    b1 = o.solve(points=pts, wpp=8, per_walk=True)
    b2 = o.solve(points=pts, wpp=8, walk_offset=8, per_walk=True)
    wa = a["walk_value"].reshape(16, 16)
    wb = np.concatenate([b1["walk_value"].reshape(16, 8), b2["walk_value"].reshape(16, 8)], 1)
    np.testing.assert_array_equal(wa, wb)
    # a subset with its original point ids reproduces those rows
    ids = np.array([3, 11, 14])
    c = o.solve(points=pts[ids], wpp=16, per_walk=True, point_ids=ids)
    np.testing.assert_array_equal(c["walk_value"].reshape(3, 16), wa[ids])
    d = o.solve(points=pts[ids], wpp=16, per_walk=True)
    assert not np.array_equal(d["walk_value"].reshape(3, 16), wa[ids])


def test_tail_recursion_reproduces_forward_sum(oracle_lib):
    """Reverse recursion V_k = c_k + w_k V_{k+1} from the terminal value gives
    back the forward walk value V_0 (the training targets' consistency)."""
    from oracle.guide_ref import tail_targets
    s = scenes.scene_c2()
    o = oracle_lib.OracleScene(s)
    for p in range(0, 2000, 173):
        tr = o.walk_trace(s.points[p], p, 3)
        V0, tails = tail_targets(tr["c"], tr["w"], tr["terminal"], killed=tr["status"] == 2)
        assert abs(V0 - tr["value"]) <= 1e-12 * max(1.0, abs(tr["value"]))
        assert tails.shape[0] == tr["c"].shape[0]


def test_roulette_is_unbiased(oracle_lib):
    """Starting roulette at step 4 with survival 0.9 keeps the C1 estimate
    unbiased (only the variance grows).  Survivor weights make the walk values
    heavy-tailed, so the check pools all points: sum of errors over its SE."""
    s = scenes.scene_c1()
    o = oracle_lib.OracleScene(s)
    pts = s.points[::4]
    r = o.solve(points=pts, wpp=512, rr_start=4, rr_q=0.9, per_walk=True)
    m, se, n = oracle_lib.estimates(r)
    err = m - _exact(s, pts)
    z_pool = err.sum() / np.sqrt(np.sum(se ** 2))
    assert abs(z_pool) < 4.5, z_pool
    assert np.any(r["walk_status"] == 2)          # roulette did kill walks
