"""The walk's Neumann-sample step (wost_neumann_sample) against brute force.

The Neumann term of a step (Sec. 3.2, eq. wost_estm) integrates
G_r(|z - x|) h(z) / alpha over the Neumann boundary inside the star.  The GPU
draws one primitive by a descent of the Neumann hierarchy and returns the
probability of its choice; the estimate is unbiased iff (i) every primitive
meeting the ball can be drawn, (ii) the returned probability is the actual
frequency of the draw, and (iii) the accepted points carry the whole
integral.  Each is checked at states on and near the boundary: the support
against the brute-force set of primitives meeting the ball, the frequencies
against the returned probabilities, and in 2D the sampled mean against an
FP64 quadrature of the integral over the visible part of the boundary in the
ball (no GPU value enters the references)."""
import numpy as np
import pytest
import torch
from scipy import stats

import scenes
from tests.gpu_common import rounded, say

pytestmark = pytest.mark.gpu

M = 1 << 16     # draws per state


@pytest.fixture(scope="module")
def W():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_18944_amd as W
    return W


@pytest.fixture(scope="module")
def O():
    import oracle
    oracle.build(force=False)
    return oracle


def _seg_closest(x, a, b):
    e = b - a
    t = np.clip(np.sum((x - a) * e, 1) / np.sum(e * e, 1), 0.0, 1.0)
    return np.linalg.norm(a + t[:, None] * e - x, axis=1)


def _visible_2d(x, zs, a, e, skip):
    """FP64: for each point z of zs, True if no segment (a, a + e) other than
    the skipped ones crosses the open segment (x, z).  Only segments meeting
    the ball can block a point inside it, so a and e hold those."""
    keep = ~skip
    a, e = a[keep], e[keep]
    if len(a) == 0:
        return np.ones(len(zs), bool)
    d = zs - x                                        # [m, 2]
    w = a[None, :, :] - x                             # [1, k, 2]
    den = d[:, None, 0] * (-e[None, :, 1]) - d[:, None, 1] * (-e[None, :, 0])
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (w[..., 0] * (-e[None, :, 1]) - w[..., 1] * (-e[None, :, 0])) / den
        u = (d[:, None, 0] * w[..., 1] - d[:, None, 1] * w[..., 0]) / den
    hit = (den != 0) & (t > 1e-12) & (t < 1 - 1e-12) & (u >= 0) & (u <= 1)
    return ~hit.any(1)


def _tri_closest(x, a, b, c):
    """FP64 distance from x to each triangle (a, b, c): to the plane where the
    foot of the perpendicular lies inside the triangle, else to the nearest
    edge."""
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    h = np.sum((x - a) * n, 1)
    p = x - h[:, None] * n
    inside = np.ones(len(a), bool)
    de_min = np.full(len(a), np.inf)
    for u, v in ((a, b), (b, c), (c, a)):
        e = v - u
        inside &= np.sum(np.cross(e, p - u) * n, 1) >= 0
        t = np.clip(np.sum((x - u) * e, 1) / np.sum(e * e, 1), 0, 1)
        de_min = np.minimum(de_min, np.linalg.norm(u + t[:, None] * e - x, axis=1))
    return np.where(inside, np.abs(h), de_min)


def _check_draws(out, support, label):
    prim = out["prim"].cpu().numpy()
    prob = out["prob"].cpu().numpy().astype(np.float64)
    drawn, cnt = np.unique(prim[prim >= 0], return_counts=True)
    assert set(drawn.tolist()) <= support, (label, set(drawn.tolist()) - support)
    # a primitive's probability is a function of the state alone
    p_of = {}
    for q in drawn:
        pq = prob[prim == q]
        assert pq.max() - pq.min() <= 1e-5 * pq.max(), (label, q, pq.min(), pq.max())
        p_of[int(q)] = float(pq.mean())
    # frequencies against the returned probabilities (chi-square over the
    # drawn primitives plus the failed draws)
    f_obs = np.array([cnt[i] for i in range(len(drawn))] + [np.sum(prim < 0)], float)
    p_exp = np.array([p_of[int(q)] for q in drawn] + [max(0.0, 1.0 - sum(p_of.values()))])
    missing = support - set(drawn.tolist())
    assert sum(p_of.values()) <= 1.0 + 1e-4, (label, sum(p_of.values()))
    if len(f_obs) > 1:
        keep = p_exp * M >= 5
        chi2 = np.sum((f_obs[keep] - M * p_exp[keep]) ** 2 / (M * p_exp[keep]))
        pval = stats.chi2.sf(chi2, max(int(keep.sum()) - 1, 1))
        assert pval > 1e-6, (label, chi2, keep.sum())
    return p_of, missing


def test_neumann_sampler_2d_against_brute_force_and_quadrature(W, O):
    """States on the outer Neumann boundary of the 2D mixed scene (all
    around, including its non-convex stretches) and just inside it, with the
    star radius of the walk (FP64 closest Dirichlet point and silhouette)."""
    s = rounded(scenes.scene_c2())
    geom = W.Geometry.from_scene(s)
    o = O.OracleScene(s)
    V, P = s.verts, s.prims
    neu = np.nonzero(s.bc == 1)[0]
    a, b = V[P[neu, 0]], V[P[neu, 1]]
    e = b - a
    meas = np.linalg.norm(e, axis=1)
    n_out = np.stack([e[:, 1], -e[:, 0]], 1) / meas[:, None]          # domain on the left of a -> b
    rng = np.random.default_rng(31)
    states = []
    for k in rng.choice(len(neu), 48, replace=False):
        t = rng.uniform(0.05, 0.95)
        states.append((np.asarray(a[k] + t * e[k], np.float32).astype(np.float64), int(neu[k]), k))
    for k in rng.choice(len(neu), 16, replace=False):
        t = rng.uniform(0.05, 0.95)
        x = a[k] + t * e[k] - 10.0 ** rng.uniform(-4, -1.5) * n_out[k]
        states.append((np.asarray(x, np.float32).astype(np.float64), -1, k))
    X = np.array([st[0] for st in states])
    Q = np.array([st[1] for st in states], np.int32)
    dD, _ = o.closest_dirichlet(X)
    dS = o.silhouette(X, on_prim=Q)
    R = np.maximum(np.minimum(dD, dS), s.eps)
    gl_s, gl_w = np.polynomial.legendre.leggauss(48)
    tau = 1e-6 * float(geom.info["diag"])
    worst = 0.0
    for i, (x, q, kq) in enumerate(states):
        r = float(np.float32(R[i]))
        d = _seg_closest(x, a, b)
        support = set(int(neu[j]) for j in np.nonzero(d < r * (1 - 1e-6))[0])
        border = set(int(neu[j]) for j in np.nonzero(np.abs(d - r) <= 1e-6 * r)[0])
        pts = torch.as_tensor(np.repeat(x[None], M, 0), dtype=torch.float32, device="cuda")
        uni = torch.as_tensor(rng.random((M, 3)), dtype=torch.float32, device="cuda")
        out = geom.neumann_sample(pts, torch.full((M,), r, dtype=torch.float32, device="cuda"), uni,
                                  on_prim=torch.full((M,), q, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        p_of, missing = _check_draws(out, support | border, "2D state %d" % i)
        assert missing <= border, ("primitives meeting the ball never drawn", i, missing)
        # sampled Neumann term with h = grad(Re z^3) . n_out
        alpha = 0.5 if q >= 0 else 1.0
        prim = out["prim"].cpu().numpy()
        ok = out["accepted"].cpu().numpy() == 1
        z = out["z"].cpu().numpy().astype(np.float64)[ok]
        jj = np.searchsorted(neu, prim[ok])
        grad = np.stack([3 * z[:, 0] ** 2 - 3 * z[:, 1] ** 2, -6 * z[:, 0] * z[:, 1]], 1)
        h = np.sum(grad * n_out[jj], 1)
        rho = np.linalg.norm(z - x, axis=1)
        prob = out["prob"].cpu().numpy().astype(np.float64)[ok]
        vals = np.zeros(M)
        vals[ok] = np.log(r / rho) / (2 * np.pi) * h * meas[jj] / prob / alpha
        est, se = vals.mean(), vals.std(ddof=1) / np.sqrt(M)
        # FP64 quadrature: each primitive's part inside the ball, split at the
        # foot of the perpendicular from x (where a boundary walker's log
        # singularity sits) with t = t_p +- (span) s^2 on each side
        nin = -n_out[kq] if q >= 0 else None
        tot = 0.0
        inball = np.nonzero(d < r)[0]
        inball_idx = inball
        for j in inball:
            A, E = a[j], e[j]
            ee = E @ E
            tp = np.clip((x - A) @ E / ee, 0.0, 1.0)
            c0 = (A - x) @ (A - x) - r * r
            disc = ((A - x) @ E) ** 2 - ee * c0
            if disc <= 0:
                continue
            t0 = max(0.0, (-(A - x) @ E - np.sqrt(disc)) / ee)
            t1 = min(1.0, (-(A - x) @ E + np.sqrt(disc)) / ee)
            for lo, hi in ((tp, t1), (tp, t0)):
                span = hi - lo
                if abs(span) < 1e-15:
                    continue
                sn = 0.5 * (gl_s + 1.0)
                t = lo + span * sn ** 2
                wq = 0.5 * gl_w * 2.0 * sn * abs(span)
                zq = A + t[:, None] * E
                dz = zq - x
                rq = np.linalg.norm(dz, axis=1)
                m = (rq < r) & (rq > 0)
                if nin is not None:
                    # the walk's tangent-plane tolerance (1e-6 of the scene
                    # diagonal): a walker's FP32 position lies up to ~1e-7
                    # off its own segment's line, whose points all count
                    m &= dz @ nin >= -tau
                m &= _visible_2d(x, zq, a[inball], e[inball], skip=(neu[inball] == q) | (inball_idx == j))
                gq = np.stack([3 * zq[:, 0] ** 2 - 3 * zq[:, 1] ** 2, -6 * zq[:, 0] * zq[:, 1]], 1) @ n_out[j]
                tot += np.sum(np.where(m, np.log(r / np.where(m, rq, 1.0)) / (2 * np.pi) * gq, 0.0) * wq) * meas[j]
        tot /= alpha
        zval = (est - tot) / max(se, 1e-12)
        worst = max(worst, abs(zval) if abs(est - tot) > 1e-4 * abs(tot) + 1e-9 else 0.0)
        assert abs(est - tot) <= 5 * se + 1e-4 * abs(tot) + 1e-9, (i, q, r, est, se, tot)
    say("2D Neumann sampler: 64 states, worst |z| of the sampled term against quadrature %.2f" % worst)


def test_neumann_sampler_3d_against_brute_force(W, O):
    """States on the Neumann half of a geodesic sphere and inside it: support
    and frequencies of the descent's choice among the triangles meeting the
    ball."""
    s = rounded(scenes.scene_halfsphere_neumann(freq=12))
    geom = W.Geometry.from_scene(s)
    o = O.OracleScene(s)
    V, P = s.verts, s.prims
    neu = np.nonzero(s.bc == 1)[0]
    A, B, C = V[P[neu, 0]], V[P[neu, 1]], V[P[neu, 2]]
    rng = np.random.default_rng(32)
    states = []
    for k in rng.choice(len(neu), 24, replace=False):
        u1, u2 = rng.uniform(0.1, 0.9, 2)
        sq = np.sqrt(u1)
        x = A[k] * (1 - sq) + B[k] * sq * (1 - u2) + C[k] * sq * u2
        states.append((np.asarray(x, np.float32).astype(np.float64), int(neu[k])))
    for _ in range(8):
        v = rng.normal(size=3)
        v[2] = abs(v[2])
        states.append((np.asarray(v / np.linalg.norm(v) * rng.uniform(0.8, 0.99), np.float32).astype(np.float64), -1))
    X = np.array([st[0] for st in states])
    Q = np.array([st[1] for st in states], np.int32)
    dD, _ = o.closest_dirichlet(X)
    dS = o.silhouette(X, on_prim=Q)
    R = np.maximum(np.minimum(np.minimum(dD, dS), 0.3), s.eps)
    for i, (x, q) in enumerate(states):
        r = float(np.float32(R[i]))
        d = _tri_closest(x, A, B, C)
        support = set(int(neu[j]) for j in np.nonzero(d < r * (1 - 1e-6))[0])
        border = set(int(neu[j]) for j in np.nonzero(np.abs(d - r) <= 1e-6 * r)[0])
        pts = torch.as_tensor(np.repeat(x[None], M, 0), dtype=torch.float32, device="cuda")
        uni = torch.as_tensor(rng.random((M, 3)), dtype=torch.float32, device="cuda")
        out = geom.neumann_sample(pts, torch.full((M,), r, dtype=torch.float32, device="cuda"), uni,
                                  on_prim=torch.full((M,), q, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        p_of, missing = _check_draws(out, support | border, "3D state %d" % i)
        assert missing <= border, ("triangles meeting the ball never drawn", i, sorted(missing)[:8])
    say("3D Neumann sampler: 32 states checked")
