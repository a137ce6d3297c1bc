"""Pins of the oracle's three-dimensional paths, and of the first star's
Neumann and source terms in both dimensions, against closed forms and
quadrature (Sec. 3.2, equation "wost_estm"; Sec. 5.3 queries).

Each pin is a ``check_*`` function that takes an oracle library handle, so
that ``test_pins_fail_under_planted_mistakes`` can run the same check against
copies of the oracle with one plausible mistake planted in them and require
it to fail.  None of these tests needs a GPU.
"""
import math
import tempfile

import numpy as np
import pytest
from scipy import integrate, special

import scenes
from tests.stats import zscore_check


def _exact(s, pts):
    from oracle import field_value
    return np.array([field_value(s.u_exact, s.dim, p) for p in pts])


def _default_lib():
    import oracle
    return oracle._load()


# ----------------------------------------------------------------------------- queries

def check_ray_cube(lib):
    """First hit from inside the axis-aligned cube [-1,1]^3 (every face
    Neumann): t = min over axes of the distance to the face ahead, and the hit
    triangle lies on that face."""
    import oracle
    s = scenes.scene_cube_box()
    s.bc[:] = 1
    o = oracle.OracleScene(s, lib=lib)
    rng = np.random.default_rng(12)
    n = 600
    x = rng.uniform(-0.9, 0.9, size=(n, 3))
    nu = rng.normal(size=(n, 3))
    nu /= np.linalg.norm(nu, axis=1, keepdims=True)
    t, prim = o.ray_neumann(x, nu, np.full(n, 10.0))
    ta = np.where(nu > 0, (1 - x) / nu, (-1 - x) / nu)          # per axis, to the face ahead
    expect = ta.min(axis=1)
    axis = ta.argmin(axis=1)
    np.testing.assert_allclose(t, expect, rtol=1e-12)
    cen = s.verts[s.prims[prim]].mean(axis=1)
    face_axis = np.argmax(np.abs(cen), axis=1)
    assert np.array_equal(face_axis, axis)
    assert np.all(np.sign(cen[np.arange(n), axis]) == np.sign(nu[np.arange(n), axis]))
    # no hit within a shorter range
    t2, p2 = o.ray_neumann(x, nu, expect * 0.999)
    assert np.all(p2 < 0) and np.all(np.isinf(t2))


def check_silhouette_convex_sphere(lib):
    """A convex closed surface has no silhouette edge seen from inside, nor
    from a point on one of its faces (that face counts as front)."""
    import oracle
    s = scenes.scene_sphere_neumann()
    o = oracle.OracleScene(s, lib=lib)
    rng = np.random.default_rng(8)
    x = rng.uniform(-0.9, 0.9, size=(1500, 3))
    x = x[np.linalg.norm(x, axis=1) < 0.9]
    assert np.all(np.isinf(o.silhouette(x)))
    q = rng.integers(0, len(s.prims), 500)
    a, b, c = (s.verts[s.prims[q, k]] for k in range(3))
    w = rng.dirichlet([1.0, 1.0, 1.0], size=500)
    on = w[:, :1] * a + w[:, 1:2] * b + w[:, 2:3] * c
    assert np.all(np.isinf(o.silhouette(on, on_prim=q)))


def check_silhouette_l_prism(lib):
    """The L-shaped prism's only silhouette seen from inside is its reflex
    edge x = y = 0 (|z| <= 1), visible as a silhouette exactly from the points
    that see one of its two faces from behind (x > 0 or y < 0); every other
    silhouette edge is farther.  Distance: sqrt(x^2 + y^2)."""
    import oracle
    o = oracle.OracleScene(scenes.scene_l_prism(), lib=lib)
    rng = np.random.default_rng(9)
    x = rng.uniform(-0.95, 0.95, size=(3000, 3))
    x = x[~((x[:, 0] > 0) & (x[:, 1] < 0))]
    x = x[(np.abs(x[:, 0]) > 1e-6) & (np.abs(x[:, 1]) > 1e-6)]
    dS = o.silhouette(x)
    hidden = (x[:, 0] <= 0) & (x[:, 1] >= 0)
    expect = np.where(hidden, np.inf, np.hypot(x[:, 0], x[:, 1]))
    assert np.array_equal(np.isinf(dS), hidden)
    np.testing.assert_allclose(dS[~hidden], expect[~hidden], rtol=1e-13)


def test_ray_axis_aligned_cube_closed_form(oracle_lib):
    check_ray_cube(_default_lib())


def test_silhouette_convex_sphere_is_empty(oracle_lib):
    check_silhouette_convex_sphere(_default_lib())


def test_silhouette_l_prism_reflex_edge_closed_form(oracle_lib):
    check_silhouette_l_prism(_default_lib())


# ----------------------------------------------------------------------------- first star

def _green(d, r, rho):
    if d == 2:
        return np.log(r / rho) / (2 * np.pi)
    return (1.0 / rho - 1.0 / r) / (4 * np.pi)


def _gauss_ball_integral(d, x, r, a, sig, c):
    """Integral over the ball B(x, r) of G_r(|y - x|) a exp(-|y - c|^2 / 2 sig^2)
    by radial quadrature of the closed-form sphere (circle) mean of the
    Gaussian."""
    D = float(np.linalg.norm(np.asarray(x) - np.asarray(c)))

    def mean_on_sphere(rho):
        if d == 2:       # (1/2pi) int exp(-(rho^2 + D^2 - 2 rho D cos t) / 2 sig^2) dt
            return math.exp(-(rho - D) ** 2 / (2 * sig ** 2)) * special.i0e(rho * D / sig ** 2)
        if D == 0.0:
            return math.exp(-rho ** 2 / (2 * sig ** 2))
        return sig ** 2 / (2 * rho * D) * (math.exp(-(rho - D) ** 2 / (2 * sig ** 2))
                                           - math.exp(-(rho + D) ** 2 / (2 * sig ** 2)))
    area = 2 * np.pi if d == 2 else 4 * np.pi
    val, _ = integrate.quad(lambda rho: area * rho ** (d - 1) * _green(d, r, rho) * mean_on_sphere(rho), 0, r,
                            limit=400, epsabs=1e-12)
    return a * val


def _mc_check(c0, expect, label, nsig=4.5):
    m = c0.mean()
    se = c0.std(ddof=1) / math.sqrt(len(c0))
    assert abs(m - expect) <= nsig * se, dict(label=label, mean=m, expect=expect, se=se, z=(m - expect) / se)
    return m, se


def check_first_step_source(lib, d):
    """Mean of the first star's source term over many walks from x equals
    -int_B G f (Sec. 3.2: the ball's Green's function; the PDE is Laplacian
    u = f), for a Gaussian f: pins the radial law of the source point
    (density proportional to G rho^(d-1)), its uniform direction, the factor
    r^2 / 2d and the sign."""
    import oracle
    # the bump is placed where the two radial laws of a plausible mistake
    # (a uniform radius) weigh it most differently: centred on x in 3D, on a
    # shell 0.3 from x in 2D
    a = 1.5
    if d == 3:
        s = scenes.scene_cube_box()
        x = np.array([0.1, -0.2, 0.05])
        c, sig = x.copy(), 0.12
    else:
        s = scenes.scene_c1()
        x = np.array([0.1, -0.2])
        c, sig = x + np.array([0.3, 0.0]), 0.1
    s.f = (scenes.FIELD["gauss_sum"], np.array([[a, sig, *c]]))
    s.g = (scenes.FIELD["zero"], np.zeros(0))
    o = oracle.OracleScene(s, lib=lib)
    r = float(o.closest_dirichlet(x[None])[0][0])
    expect = -_gauss_ball_integral(d, x, r, a, sig, c)
    c0 = o.first_step(x, 200000, p=3)
    return _mc_check(c0, expect, "source d=%d" % d) + (expect,)


def _disk_green_integral(h0, R, r):
    """int over the disk of radius R at height h0 above x of G_r(distance), 3D."""
    val, _ = integrate.quad(lambda s: 2 * np.pi * s * _green(3, r, math.sqrt(h0 * h0 + s * s)), 0, R,
                            limit=200, epsabs=1e-12)
    return val


def check_first_step_neumann(lib):
    """Mean of the first star's Neumann term from x (off the boundary) equals
    int over the Neumann part inside the ball of G h (Sec. 3.2): the ball
    around x meets the cube's Neumann face y = 1 in a disk, h = du/dn_out =
    -2 there.  Pins the point drawn on a triangle, the area weight, the 3D
    Green's function and the orientation of h."""
    import oracle
    s = scenes.scene_cube_neumann_face()
    s.g = (scenes.FIELD["zero"], np.zeros(0))
    o = oracle.OracleScene(s, lib=lib)
    x = np.array([0.1, 0.5, -0.05])
    r = 0.9                                  # nearest Dirichlet face x = 1; the face's rim is farther
    assert abs(o.closest_dirichlet(x[None])[0][0] - r) < 1e-14
    assert o.silhouette(x[None])[0] > r
    h0 = 1.0 - x[1]
    R = math.sqrt(r * r - h0 * h0)
    expect = -2.0 * _disk_green_integral(h0, R, r)
    c0 = o.first_step(x, 200000, p=5)
    return _mc_check(c0, expect, "neumann 3D") + (expect,)


@pytest.mark.parametrize("d", [2, 3])
def test_first_star_source_term_matches_green_integral(oracle_lib, d):
    check_first_step_source(_default_lib(), d)


def test_first_star_neumann_term_matches_green_integral(oracle_lib):
    check_first_step_neumann(_default_lib())


# ----------------------------------------------------------------------------- estimator in 3D

def _eps_allow(s, pts, grad_max):
    return np.full(len(pts), s.eps * grad_max)


def check_half_neumann_cube(lib, wpp=1024):
    """Cube with its face y = 1 Neumann (h = -2 from u = x^2 - y^2), other
    faces Dirichlet: the estimate matches u per point (walkers reflect on
    the Neumann face, alpha = 1/2 there)."""
    import oracle
    s = scenes.scene_cube_neumann_face()
    o = oracle.OracleScene(s, lib=lib)
    r = o.solve(wpp=wpp)
    m, se, n = oracle.estimates(r)
    return zscore_check(m, se, _exact(s, s.points), n, label="half-Neumann cube",
                        allow=_eps_allow(s, s.points, 2 * math.sqrt(2)))


def check_half_neumann_sphere(lib, wpp=256):
    """Unit geodesic sphere, upper half Neumann with h = grad(x^2 - y^2).n_out,
    lower half Dirichlet: curved Neumann surface, silhouettes along the rim,
    rays and visibility on triangles."""
    import oracle
    s = scenes.scene_halfsphere_neumann()
    o = oracle.OracleScene(s, lib=lib)
    r = o.solve(wpp=wpp)
    m, se, n = oracle.estimates(r)
    return zscore_check(m, se, _exact(s, s.points), n, label="half-Neumann sphere",
                        allow=_eps_allow(s, s.points, 2.0))


def check_cube_poisson(lib, wpp=256):
    """Manufactured u = |x|^2 (Laplacian u = 6) on the cube: the 3D source
    term's sign and factor r^2 / 2d."""
    import oracle
    s = scenes.scene_cube_poisson()
    o = oracle.OracleScene(s, lib=lib)
    r = o.solve(wpp=wpp)
    m, se, n = oracle.estimates(r)
    info = zscore_check(m, se, _exact(s, s.points), n, label="cube Poisson",
                        allow=_eps_allow(s, s.points, 2 * math.sqrt(3)))
    # a flipped sign would be off by 2 (E[sum of r^2]) ~ 2 (1 - |x|^2 / 3) on average
    assert np.mean(np.abs(m - _exact(s, s.points))) < 0.05
    return info


def test_half_neumann_cube_matches_closed_form(oracle_lib):
    check_half_neumann_cube(_default_lib())


def test_half_neumann_sphere_matches_closed_form(oracle_lib):
    check_half_neumann_sphere(_default_lib())


def test_cube_poisson_pins_3d_source(oracle_lib):
    check_cube_poisson(_default_lib())


# ----------------------------------------------------------------------------- planted mistakes

# (name, text in the oracle source, replacement, checks that must fail)
MUTANTS = [
    ("triangle point without the square root", "double sq = sqrt(u[1]);", "double sq = u[1];",
     ["neumann3"]),
    ("3D source radius uniform instead of Beta(2,2)", "sr = fmax(fmin(a, b), fmin(fmax(a, b), c));",
     "sr = a;", ["source3"]),
    ("2D source radius uniform instead of sqrt(U1 U2)", "sr = sqrt(ua[0] * ua[1]);", "sr = ua[0];",
     ["source2"]),
    ("source sign flipped", "contrib += -(r * r / (2.0 * d))", "contrib += (r * r / (2.0 * d))",
     ["source3", "poisson3"]),
    ("3D ray distance from the wrong edge", "return dot(3, e2, qv) / det;", "return dot(3, e1, qv) / det;",
     ["ray3"]),
    ("3D silhouette distance to an edge's first vertex only", "closest_on_segment(3, x, P, P + 3, tmp)",
     "closest_on_segment(3, x, P, P, tmp)", ["sil3"]),
    ("3D Green's function normalised by 2 pi", "return (1.0 / rho - 1.0 / r) / (4.0 * OR_PI);",
     "return (1.0 / rho - 1.0 / r) / (2.0 * OR_PI);", ["neumann3", "poisson3"]),
    ("Neumann term without 1 / alpha", "contrib += green_ball(d, r, rho) * hv * A / alpha;",
     "contrib += green_ball(d, r, rho) * hv * A;", ["cube_neumann"]),
    ("Neumann data with the inward sign", "contrib += green_ball(d, r, rho) * hv * A / alpha;",
     "contrib -= green_ball(d, r, rho) * hv * A / alpha;", ["neumann3", "cube_neumann"]),
]

CHECKS = {
    "ray3": check_ray_cube,
    "sil3": check_silhouette_l_prism,
    "source2": lambda lib: check_first_step_source(lib, 2),
    "source3": lambda lib: check_first_step_source(lib, 3),
    "neumann3": check_first_step_neumann,
    "cube_neumann": lambda lib: check_half_neumann_cube(lib, wpp=256),
    "poisson3": lambda lib: check_cube_poisson(lib, wpp=64),
}


@pytest.mark.parametrize("name,find,repl,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_fail_under_planted_mistakes(oracle_lib, name, find, repl, checks):
    """Each pin above must catch the mistake it is meant for: a copy of the
    oracle with that one change planted (on the CPU) fails the named check."""
    import oracle
    src = oracle.source_text()
    assert src.count(find) == 1, "planted-mistake anchor not found once: %r" % find
    with tempfile.TemporaryDirectory() as tmp:
        lib = oracle.load_variant(src.replace(find, repl), tmp, "m")
        for c in checks:
            with pytest.raises(AssertionError):
                CHECKS[c](lib)
