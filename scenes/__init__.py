"""Seeded synthetic scenes for guided walk-on-stars (WoSt).

This module only *generates inputs*: boundary polylines / triangle meshes with a
per-primitive boundary-condition tag, analytic boundary-data descriptors and
query points.  It holds none of the estimator's arithmetic (no distances,
normals, Green's functions or sampling), so that the FP64 oracle and the HIP
path can both consume the same arrays without sharing any method code.

Conventions of the produced data
--------------------------------
* 2D: ``prims[i] = (a, b)`` is a directed segment; the domain lies to the
  LEFT of a->b (outer boundary counter-clockwise, holes clockwise).
* 3D: ``prims[i] = (a, b, c)`` is wound so that (b-a)x(c-a) points OUT of the
  domain (outer surface: away from the origin; holes: towards their centre).
* ``bc[i]`` is 0 for a Dirichlet primitive and 1 for a Neumann primitive.
* Boundary data are given by field descriptors ``(kind, params)`` whose kinds
  are the integer codes in :data:`FIELD`; a Neumann descriptor of a potential
  kind means h = grad(phi).n_out (outward normal derivative).

The problem statement these scenes instantiate is the mixed Poisson problem of
the paper's background section (Poisson equation with Dirichlet and Neumann
boundary conditions); the shapes and sizes follow the synthetic stand-ins for
the paper's mesh and diffusion-curve datasets (Sec. 6).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

# Analytic field kinds (shared integer codes; evaluation is done by each side).
FIELD = {
    "zero": 0,        # 0
    "const": 1,       # params[0]
    "exp_sin": 2,     # e^x sin y                       (harmonic, 2D)
    "re_z3": 3,       # Re z^3 = x^3 - 3 x y^2          (harmonic, 2D)
    "x2_minus_y2": 4,  # x^2 - y^2                       (harmonic, 2D/3D)
    "r2": 5,          # |x|^2                           (Laplacian 2d)
    "gauss_sum": 6,   # sum_j a_j exp(-|x-c_j|^2/(2 s_j^2)); params rows (a, s, c_1..c_d)
}

SCENE_SEED = 2410
WALK_SEED = 18944


@dataclasses.dataclass
class Scene:
    name: str
    dim: int
    verts: np.ndarray          # float64 [n_verts, dim]
    prims: np.ndarray          # int32 [n_prims, dim]
    bc: np.ndarray             # uint8 [n_prims]
    points: np.ndarray         # float64 [n_points, dim]
    g: tuple                   # (kind, params float64[...]) Dirichlet value
    h: tuple                   # (kind, params) Neumann data (outward derivative)
    f: tuple                   # (kind, params) source, Laplacian u = f
    u_exact: tuple | None      # (kind, params) closed-form solution, if any
    eps: float = 1e-3
    max_steps: int = 4096
    rr_start: int = 128
    rr_q: float = 0.99
    wpp: int = 64
    meta: dict = dataclasses.field(default_factory=dict)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.verts, self.prims, self.bc, self.points):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    def subset(self, idx) -> "Scene":
        s = dataclasses.replace(self)
        s.points = np.ascontiguousarray(self.points[idx])
        return s


def _zero():
    return (FIELD["zero"], np.zeros(0))


def _kind(name):
    return (FIELD[name], np.zeros(0))


# ----------------------------------------------------------------------------
# 2D generators
# ----------------------------------------------------------------------------

def _circle(n, cx, cy, r, ccw=True):
    t = 2.0 * np.pi * np.arange(n) / n
    if not ccw:
        t = -t
    return np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], axis=1)


def _loop_prims(offset, n):
    i = np.arange(n, dtype=np.int64)
    return np.stack([offset + i, offset + (i + 1) % n], axis=1).astype(np.int32)


def _point_in_polygon(px, py, poly):
    """Even-odd crossing test (input filtering only)."""
    inside = np.zeros(px.shape, dtype=bool)
    x0, y0 = poly[:, 0], poly[:, 1]
    x1, y1 = np.roll(x0, -1), np.roll(y0, -1)
    for a0, b0, a1, b1 in zip(x0, y0, x1, y1):
        cond = (b0 > py) != (b1 > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xc = a0 + (py - b0) * (a1 - a0) / (b1 - b0)
        inside ^= cond & (px < xc)
    return inside


def scene_c1(wpp: int = 64) -> Scene:
    """Unit disk as a 128-gon, all Dirichlet, g = e^x sin y; 32x32 lattice of
    cell centres on [-0.9, 0.9]^2 restricted to r < 0.9."""
    verts = _circle(128, 0.0, 0.0, 1.0, ccw=True)
    prims = _loop_prims(0, 128)
    bc = np.zeros(128, np.uint8)
    c = -0.9 + (np.arange(32) + 0.5) * (1.8 / 32)
    X, Y = np.meshgrid(c, c, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    P = P[np.hypot(P[:, 0], P[:, 1]) < 0.9]
    return Scene("C1", 2, verts, prims, bc, np.ascontiguousarray(P),
                 g=_kind("exp_sin"), h=_zero(), f=_zero(), u_exact=_kind("exp_sin"),
                 eps=1e-3, max_steps=256, rr_start=1 << 30, rr_q=1.0, wpp=wpp,
                 meta={"n_outer": 128})


def scene_c1_poisson(wpp: int = 64) -> Scene:
    """C1 geometry with the manufactured solution u = |x|^2 (Laplacian = 4)."""
    s = scene_c1(wpp)
    s = dataclasses.replace(s, name="C1-poisson", g=_kind("r2"),
                            f=(FIELD["const"], np.array([4.0])), u_exact=_kind("r2"))
    return s


def _star_polygon(rng, n, n_modes=8, amp=0.2):
    a = rng.standard_normal(n_modes) / np.arange(1, n_modes + 1)
    b = rng.standard_normal(n_modes) / np.arange(1, n_modes + 1)
    th = 2.0 * np.pi * np.arange(n) / n
    m = np.arange(1, n_modes + 1)
    pert = (np.cos(np.outer(th, m)) @ a) + (np.sin(np.outer(th, m)) @ b)
    pert *= amp / np.max(np.abs(pert))
    r = 1.0 + pert
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1), r


def scene_c2(seed: int = SCENE_SEED, n_outer: int = 4096, n_hole: int = 256,
             n_holes: int = 4, grid: int = 256, wpp: int = 256) -> Scene:
    """Seeded star-shaped outer polygon (Neumann, u = Re z^3 data) with
    circular Dirichlet holes; lattice of query points over the outer AABB."""
    rng = np.random.default_rng(seed)
    outer, r_outer = _star_polygon(rng, n_outer)
    r_min = float(r_outer.min())
    holes = []
    tries = 0
    while len(holes) < n_holes:
        tries += 1
        if tries > 100000:
            raise RuntimeError("hole placement failed")
        rh = rng.uniform(0.1, 0.2)
        c = rng.uniform(-0.8, 0.8, size=2)
        if np.hypot(*c) + rh + 0.05 > r_min:
            continue
        if any(np.hypot(*(c - c2)) < rh + r2 + 0.05 for c2, r2 in holes):
            continue
        holes.append((c, rh))
    verts = [outer]
    prims = [_loop_prims(0, n_outer)]
    bc = [np.ones(n_outer, np.uint8)]
    off = n_outer
    for c, rh in holes:
        verts.append(_circle(n_hole, c[0], c[1], rh, ccw=False))
        prims.append(_loop_prims(off, n_hole))
        bc.append(np.zeros(n_hole, np.uint8))
        off += n_hole
    verts = np.concatenate(verts)
    prims = np.concatenate(prims)
    bc = np.concatenate(bc)
    lo = outer.min(axis=0)
    hi = outer.max(axis=0)
    cx = lo[0] + (np.arange(grid) + 0.5) * (hi[0] - lo[0]) / grid
    cy = lo[1] + (np.arange(grid) + 0.5) * (hi[1] - lo[1]) / grid
    X, Y = np.meshgrid(cx, cy, indexing="xy")
    px, py = X.ravel(), Y.ravel()
    keep = _point_in_polygon(px, py, outer)
    for c, rh in holes:
        keep &= np.hypot(px - c[0], py - c[1]) > rh + 2e-3
    P = np.ascontiguousarray(np.stack([px[keep], py[keep]], axis=1))
    return Scene("C2", 2, verts, prims, bc, P,
                 g=_kind("re_z3"), h=_kind("re_z3"), f=_zero(), u_exact=_kind("re_z3"),
                 eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99, wpp=wpp,
                 meta={"holes": [(c.tolist(), rh) for c, rh in holes],
                       "grid": grid, "n_outer": n_outer, "n_hole": n_hole,
                       "aabb": [lo.tolist(), hi.tolist()]})


def scene_halfdisk_neumann(n: int = 256, wpp: int = 64) -> Scene:
    """Unit disk, upper arc Neumann / lower arc Dirichlet, u = Re z^3.
    Small mixed problem that pins the sign convention of the Neumann data."""
    verts = _circle(n, 0.0, 0.0, 1.0, ccw=True)
    prims = _loop_prims(0, n)
    mid = 0.5 * (verts[prims[:, 0]] + verts[prims[:, 1]])
    bc = (mid[:, 1] > 0).astype(np.uint8)
    c = -0.8 + (np.arange(8) + 0.5) * (1.6 / 8)
    X, Y = np.meshgrid(c, c, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    P = P[np.hypot(P[:, 0], P[:, 1]) < 0.8]
    return Scene("halfdisk", 2, verts, prims, bc, np.ascontiguousarray(P),
                 g=_kind("re_z3"), h=_kind("re_z3"), f=_zero(), u_exact=_kind("re_z3"),
                 eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99, wpp=wpp)


# ----------------------------------------------------------------------------
# 3D generators
# ----------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], float)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    return v / np.linalg.norm(v, axis=1, keepdims=True), f


def geodesic_sphere(freq: int):
    """Class-I geodesic subdivision of the icosahedron: 20*freq^2 triangles on
    the unit sphere, outward winding, shared vertices merged."""
    v0, f0 = _icosahedron()
    # integer barycentric lattice per face; global vertex key from the exact
    # rational position (i*A + j*B + k*C)/freq expressed on icosahedron ids
    keys = {}
    pos = []
    tri = []

    def vid(ids_w):
        # ids_w: tuple of (vertex id, weight) with weights summing to freq
        key = tuple(sorted((a, w) for a, w in ids_w if w > 0))
        j = keys.get(key)
        if j is None:
            j = len(pos)
            keys[key] = j
            p = sum(w * v0[a] for a, w in key) / freq
            pos.append(p)
        return j

    for A, B, C in f0:
        idx = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                k = freq - i - j
                idx[(i, j)] = vid(((A, k), (B, i), (C, j)))
        for i in range(freq):
            for j in range(freq - i):
                a = idx[(i, j)]
                b = idx[(i + 1, j)]
                c = idx[(i, j + 1)]
                tri.append((a, b, c))
                if j + 1 <= freq - i - 1:
                    d = idx[(i + 1, j + 1)]
                    tri.append((b, d, c))
    P = np.asarray(pos)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    T = np.asarray(tri, np.int64)
    # orient outward
    n = np.cross(P[T[:, 1]] - P[T[:, 0]], P[T[:, 2]] - P[T[:, 0]])
    flip = np.einsum("ij,ij->i", n, P[T].mean(axis=1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return P, T.astype(np.int32)


def _radial_field(rng, n_waves=16, amp=0.15):
    k_dir = rng.standard_normal((n_waves, 3))
    k_dir /= np.linalg.norm(k_dir, axis=1, keepdims=True)
    k = k_dir * rng.uniform(1.0, 4.0, size=(n_waves, 1))
    phi = rng.uniform(0, 2 * np.pi, size=n_waves)

    def raw(p):
        return np.cos(p @ k.T + phi).sum(axis=1)
    return raw, amp


def scene_3d(name: str, freq: int, seed: int = SCENE_SEED, hole_level_freq: int = 16,
             slice_grid: int | None = 512, n_random: int | None = None,
             wpp: int = 1024, with_source: bool = False) -> Scene:
    rng = np.random.default_rng(seed + freq)
    P, T = geodesic_sphere(freq)
    raw, amp = _radial_field(rng)
    d = raw(P)
    A = amp / np.max(np.abs(d))
    P = P * (1.0 + A * d)[:, None]
    r_in = float(np.linalg.norm(P, axis=1).min())

    def R_of(u):
        return 1.0 + A * raw(u)

    hv, ht = geodesic_sphere(hole_level_freq)
    holes = []
    tries = 0
    while len(holes) < 3:
        tries += 1
        if tries > 100000:
            raise RuntimeError("hole placement failed")
        rh = rng.uniform(0.1, 0.2)
        c = rng.uniform(-0.6, 0.6, size=3)
        if not holes:
            c[2] = rng.uniform(-0.5 * rh, 0.5 * rh)   # first hole crosses z = 0
        if np.linalg.norm(c) + rh + 0.05 > r_in:
            continue
        if any(np.linalg.norm(c - c2) < rh + r2 + 0.05 for c2, r2 in holes):
            continue
        holes.append((c, rh))
    verts = [P]
    prims = [T]
    cen = P[T].mean(axis=1)
    bc = [(cen[:, 2] > 0).astype(np.uint8)]
    off = P.shape[0]
    for c, rh in holes:
        verts.append(c + rh * hv)
        prims.append((ht[:, [0, 2, 1]] + off).astype(np.int32))  # inward = out of domain
        bc.append(np.zeros(ht.shape[0], np.uint8))
        off += hv.shape[0]
    verts = np.concatenate(verts)
    prims = np.concatenate(prims).astype(np.int32)
    bc = np.concatenate(bc)
    lo, hi = P.min(axis=0), P.max(axis=0)

    def keep_mask(Q):
        rq = np.linalg.norm(Q, axis=1)
        u = Q / np.maximum(rq, 1e-300)[:, None]
        m = rq < R_of(u) - 0.01
        for c, rh in holes:
            m &= np.linalg.norm(Q - c, axis=1) > rh + 2e-3
        return m

    if n_random is None:
        g = slice_grid
        cx = lo[0] + (np.arange(g) + 0.5) * (hi[0] - lo[0]) / g
        cy = lo[1] + (np.arange(g) + 0.5) * (hi[1] - lo[1]) / g
        X, Y = np.meshgrid(cx, cy, indexing="xy")
        Q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
        Q = Q[keep_mask(Q)]
    else:
        out = []
        need = n_random
        prng = np.random.default_rng(seed + 7)
        while need > 0:
            Qc = prng.uniform(lo, hi, size=(max(2 * need, 1024), 3))
            Qc = Qc[keep_mask(Qc)][:need]
            out.append(Qc)
            need -= Qc.shape[0]
        Q = np.concatenate(out)
    f = _zero()
    if with_source:
        srng = np.random.default_rng(seed + 11)
        rows = []
        while len(rows) < 16:
            cpos = srng.uniform(-0.7, 0.7, size=3)
            if not keep_mask(cpos[None])[0]:
                continue
            rows.append([srng.uniform(0.5, 2.0), srng.uniform(0.05, 0.2), *cpos])
        f = (FIELD["gauss_sum"], np.asarray(rows, float))
    return Scene(name, 3, np.ascontiguousarray(verts), prims, bc, np.ascontiguousarray(Q),
                 g=_kind("x2_minus_y2"), h=_kind("x2_minus_y2"), f=f,
                 u_exact=None if with_source else _kind("x2_minus_y2"),
                 eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99, wpp=wpp,
                 meta={"holes": [(c.tolist(), rh) for c, rh in holes], "freq": freq})


def scene_c4(freq: int = 100, **kw) -> Scene:
    return scene_3d("C4", freq, **kw)


def scene_c5(freq: int = 224, n_random: int = 1 << 20, **kw) -> Scene:
    return scene_3d("C5", freq, n_random=n_random, with_source=True, **kw)


def scene_c5_manufactured(n_random: int = 8192, freq: int = 224, **kw) -> Scene:
    """The C5 geometry (noise-displaced sphere with three holes, z > 0 of the
    outer surface Neumann) with the manufactured solution u = |x|^2: source
    Laplacian u = 6, Dirichlet g = u, Neumann data its outward derivative;
    n_random uniform interior query points."""
    s = scene_3d("C5-manufactured", freq, n_random=n_random, **kw)
    return dataclasses.replace(s, g=_kind("r2"), h=_kind("r2"), f=(FIELD["const"], np.array([6.0])),
                               u_exact=_kind("r2"))


def scene_sphere_sources(freq: int = 6, n_points: int = 64, wpp: int = 64, seed: int = 12) -> Scene:
    """Geodesic unit sphere, all Dirichlet with g = x^2 - y^2, and a source
    of 16 seeded Gaussian bumps (amplitudes U(0.5, 2), widths U(0.05, 0.2),
    centres in the ball r < 0.7) -- the source recipe of the 1M-triangle
    Poisson workload on a mesh small enough for brute-force queries."""
    V, T = geodesic_sphere(freq)
    rng = np.random.default_rng(seed)
    rows = []
    while len(rows) < 16:
        c = rng.uniform(-0.7, 0.7, size=3)
        if np.linalg.norm(c) < 0.7:
            rows.append([rng.uniform(0.5, 2.0), rng.uniform(0.05, 0.2), *c])
    Q = rng.uniform(-0.8, 0.8, size=(8 * n_points, 3))
    Q = Q[np.linalg.norm(Q, axis=1) < 0.8][:n_points]
    return Scene("sphere-sources", 3, V, T, np.zeros(T.shape[0], np.uint8), np.ascontiguousarray(Q),
                 g=_kind("x2_minus_y2"), h=_zero(), f=(FIELD["gauss_sum"], np.asarray(rows, float)),
                 u_exact=None, eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99, wpp=wpp)


def scene_cube_box(wpp: int = 64) -> Scene:
    """Axis-aligned unit cube [-1,1]^3 (12 triangles), all Dirichlet, u = x^2 - y^2."""
    v = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], float)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    tri = []
    for a, b, c, d in quads:
        tri += [(a, b, c), (a, c, d)]
    T = np.asarray(tri, np.int64)
    n = np.cross(v[T[:, 1]] - v[T[:, 0]], v[T[:, 2]] - v[T[:, 0]])
    flip = np.einsum("ij,ij->i", n, v[T].mean(axis=1)) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    rng = np.random.default_rng(5)
    Q = rng.uniform(-0.8, 0.8, size=(64, 3))
    return Scene("cube", 3, v, T.astype(np.int32), np.zeros(12, np.uint8), Q,
                 g=_kind("x2_minus_y2"), h=_zero(), f=_zero(), u_exact=_kind("x2_minus_y2"),
                 eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99, wpp=wpp)


def scene_cube_neumann_face(wpp: int = 256) -> Scene:
    """Cube [-1,1]^3 whose face y = +1 (two large triangles) is Neumann with
    the outward derivative of u = x^2 - y^2 (h = -2 there); the other faces
    are Dirichlet with g = u.  Large flat Neumann triangles make the
    estimate sensitive to how points are drawn on them."""
    s = scene_cube_box(wpp)
    cen = s.verts[s.prims].mean(axis=1)
    bc = (cen[:, 1] > 0.99).astype(np.uint8)
    return dataclasses.replace(s, name="cube-neumann-face", bc=bc, h=_kind("x2_minus_y2"))


def scene_cube_poisson(wpp: int = 256) -> Scene:
    """Cube [-1,1]^3, all Dirichlet, manufactured u = |x|^2 (Laplacian u = 6)."""
    s = scene_cube_box(wpp)
    return dataclasses.replace(s, name="cube-poisson", g=_kind("r2"), f=(FIELD["const"], np.array([6.0])),
                               u_exact=_kind("r2"))


def scene_halfsphere_neumann(freq: int = 6, n_points: int = 64, wpp: int = 256, seed: int = 6) -> Scene:
    """Geodesic unit sphere (20 freq^2 triangles): faces with centroid z > 0
    Neumann with the outward derivative of u = x^2 - y^2, the others
    Dirichlet with g = u; query points uniform in the ball r < 0.8."""
    V, T = geodesic_sphere(freq)
    cen = V[T].mean(axis=1)
    bc = (cen[:, 2] > 0).astype(np.uint8)
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-0.8, 0.8, size=(4 * n_points, 3))
    Q = Q[np.linalg.norm(Q, axis=1) < 0.8][:n_points]
    return Scene("halfsphere", 3, V, T, bc, np.ascontiguousarray(Q), g=_kind("x2_minus_y2"),
                 h=_kind("x2_minus_y2"), f=_zero(), u_exact=_kind("x2_minus_y2"),
                 eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99, wpp=wpp)


def scene_sphere_neumann(freq: int = 6) -> Scene:
    """Geodesic unit sphere, every face Neumann (a convex closed surface)."""
    V, T = geodesic_sphere(freq)
    return Scene("sphere-neumann", 3, V, T, np.ones(T.shape[0], np.uint8), np.zeros((1, 3)),
                 g=_zero(), h=_zero(), f=_zero(), u_exact=None)


def scene_l_prism() -> Scene:
    """L-shaped prism: the square [-1,1]^2 without the quadrant x > 0, y < 0,
    extruded over z in [-1, 1]; every face Neumann.  Its one reflex edge is
    the segment x = y = 0, |z| <= 1.  Side quads are split along a diagonal,
    the end caps fanned from the reflex corner."""
    L2 = np.array([[-1, -1], [0, -1], [0, 0], [1, 0], [1, 1], [-1, 1]], float)   # counter-clockwise
    n = L2.shape[0]
    V = np.concatenate([np.c_[L2, -np.ones(n)], np.c_[L2, np.ones(n)]])
    T = []
    for i in range(n):
        j = (i + 1) % n
        a, b, c, d = i, j, n + j, n + i           # side quad, counter-clockwise seen from outside
        T += [(a, b, c), (a, c, d)]
    for k in (3, 4, 5, 0):                         # caps: fan from the reflex corner (vertex 2)
        T.append((n + 2, n + k, n + (k + 1) % n))  # top, outward +z
        T.append((2, (k + 1) % n, k))              # bottom, outward -z
    T = np.asarray(T, np.int32)
    return Scene("l-prism", 3, V, T, np.ones(T.shape[0], np.uint8), np.zeros((1, 3)),
                 g=_zero(), h=_zero(), f=_zero(), u_exact=None)


SCENES = {
    "C1": scene_c1,
    "C1-poisson": scene_c1_poisson,
    "C2": scene_c2,
    "halfdisk": scene_halfdisk_neumann,
    "C4": scene_c4,
    "C5": scene_c5,
    "cube": scene_cube_box,
    "cube-neumann-face": scene_cube_neumann_face,
    "cube-poisson": scene_cube_poisson,
    "halfsphere": scene_halfsphere_neumann,
    "C5-manufactured": scene_c5_manufactured,
    "sphere-sources": scene_sphere_sources,
}


def make_scene(name: str, **kw) -> Scene:
    return SCENES[name](**kw)
