"""Per-point parity of the GPU estimators with closed forms and the FP64
oracle on the benchmark workloads, through the paths the benchmark times.

* Russian roulette (Sec. 6.1: from step 128 in the paper; here from step 4
  with survival 0.9 so that it fires on most walks) walk by walk against the
  oracle on the same Philox words, and unbiased against the closed form.
* The 2D mixed workload (43,347 points): every point's estimate within 3 of
  its standard errors of Re z^3 -- at the benchmark's 256 walks per point,
  uniform and with the online-trained guide (the benchmark's schedule:
  16-walk batches, training through 64 walks per point, then inference
  only), and uniform at 16,384 walks per point, where biases of 1e-3 show.
* The 3D workloads at full geometric size on seeded samples of points:
  x^2 - y^2 on the 215k-triangle mesh (uniform and online-guided), and the
  manufactured Poisson solution |x|^2 on the 1M-triangle mesh (source term
  and mixed boundaries), per point against the closed form.
* The 3D source term walk by walk against the oracle (Gaussian-bump source of
  the 1M-triangle workload on a mesh small enough for brute force).

The statistical criterion is that of tests/stats.py (exceedances of |z| > 3
against the binomial tail, mean and variance of z).  Every comparison allows
the epsilon-shell bias eps * sup |grad u| over the Dirichlet boundary per
point (a walk ends at distance <= eps and scores g at the closest point)."""
import dataclasses

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_common import exact_solution, rounded, say
from tests.stats import two_sample_z, zscore_check

pytestmark = pytest.mark.gpu

RR_Q = float(np.float32(0.9))     # both sides decide roulette against the same FP32 value


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


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float32), device="cuda")


def _solve(W, geom, s, pts, wpp, seed, per_walk=False, guide=None, **pkw):
    pb = W.Problem.from_scene(s, **pkw)
    n = pts.shape[0]
    wv = torch.empty(n * wpp, dtype=torch.float32, device="cuda") if per_walk else None
    ws = torch.empty(n * wpp, dtype=torch.int32, device="cuda") if per_walk else None
    acc = W.solve(geom, pb, pts, wpp, seed=seed, guide=guide, walk_value=wv, walk_steps=ws)
    torch.cuda.synchronize()
    m, se, cnt = acc.estimates()
    out = dict(mean=m.cpu().numpy(), se=se.cpu().numpy(), n=cnt.cpu().numpy(), stats=acc.stats(),
               var=(se.cpu().numpy() ** 2) * cnt.cpu().numpy())
    if per_walk:
        out.update(walk_value=wv.double().cpu().numpy(), walk_steps=ws.cpu().numpy())
    return out


def _online(W, geom, s, pts, wpp, seed, guide_seed, batch_wpp=16, train_until=64):
    from paper_2410_18944_amd.driver import OnlineSchedule, online_solve
    g = W.Guide(W.GuideConfig.for_scene(s), seed=guide_seed)
    pb = W.Problem.from_scene(s, sampling="mis_learned")
    sched = OnlineSchedule(batch_wpp=batch_wpp, train_until_wpp=train_until)
    acc, info = online_solve(geom, pb, pts, wpp, g, sched, seed=seed)
    m, se, cnt = acc.estimates()
    return dict(mean=m.cpu().numpy(), se=se.cpu().numpy(), n=cnt.cpu().numpy(), stats=acc.stats(),
                var=(se.cpu().numpy() ** 2) * cnt.cpu().numpy(), info=info)


def _dirichlet_grad_bound(s, grad_norm):
    """eps * sup |grad u| over the Dirichlet boundary (vertices of Dirichlet
    primitives, which bound |grad u| on them for these polynomial u)."""
    dv = np.unique(s.prims[s.bc == 0])
    return s.eps * float(np.max(grad_norm(s.verts[dv])))


def _grad_re_z3(p):
    return 3.0 * (p[:, 0] ** 2 + p[:, 1] ** 2)


def _grad_x2_y2(p):
    return 2.0 * np.hypot(p[:, 0], p[:, 1])


def _grad_r2(p):
    return 2.0 * np.linalg.norm(p, axis=1)


def _check_run(r, n_walks):
    st = r["stats"]
    assert st["walks"] == n_walks, st
    assert st["nonfinite"] == 0 and st["truncated"] == 0, st


# ----------------------------------------------------------------------------- Russian roulette

@pytest.mark.parametrize("name", ["C1", "cube", "cube-poisson", "C2"])
def test_roulette_walk_by_walk_against_the_oracle(W, O, name):
    """Roulette from step 4 with survival 0.9: the GPU plays it at the end of
    step k-1 with the fourth word of step k's Neumann block, the oracle at the
    start of step k with the same word -- the same event, so walks end at the
    same step, and the weight 1/q of survivors gives the same values."""
    s = rounded(scenes.make_scene(name))
    s.max_steps = 4096
    s.rr_start, s.rr_q = 4, RR_Q
    wpp = 64 if name != "C2" else 32
    pts = s.points if name != "C2" else s.points[::97][:256]
    say("roulette walk by walk:", name, len(pts), "points x", wpp)
    geom = W.Geometry.from_scene(s)
    g = _solve(W, geom, s, _t(pts), wpp, 18944, per_walk=True)
    o = O.OracleScene(s).solve(points=pts, wpp=wpp, per_walk=True)
    same = g["walk_steps"] == o["walk_steps"]
    kills_o = int(np.sum(o["walk_status"] == 2))
    say("  identical step counts %.4f; roulette kills GPU %d oracle %d" % (same.mean(), g["stats"]["rr_killed"],
                                                                          kills_o))
    assert kills_o > 0.2 * len(pts) * wpp
    assert same.mean() > 0.99, same.mean()
    assert abs(g["stats"]["rr_killed"] - kills_o) <= 0.01 * kills_o + 2
    if name != "C2":
        # Dirichlet-only scenes: the walk value is unique given its words
        dv = np.abs(g["walk_value"] - o["walk_value"])[same]
        tol = 1e-4 * np.maximum(1.0, np.abs(o["walk_value"][same]))
        assert np.mean(dv <= tol) > 0.995, np.percentile(dv, [50, 99, 100])
    else:
        # Neumann points are drawn by different valid samplers on the two sides
        mo, so, _ = O.estimates(o)
        z = two_sample_z(g["mean"], g["se"], mo, so)
        assert np.mean(np.abs(z) > 3) < 0.02 and abs(z.mean()) < 5 / np.sqrt(len(z)), z


def test_roulette_is_unbiased_against_the_closed_form(W):
    s = scenes.scene_c1()
    s.rr_start, s.rr_q = 4, RR_Q
    say("C1 with roulette from step 4, 2048 wpp")
    geom = W.Geometry.from_scene(s)
    g = _solve(W, geom, s, _t(s.points), 2048, 7)
    assert g["stats"]["rr_killed"] > 0.2 * s.n_points * 2048
    zscore_check(g["mean"], g["se"], exact_solution(s, s.points), g["n"], label="C1 roulette")


# ----------------------------------------------------------------------------- 2D mixed workload, full grid

@pytest.fixture(scope="module")
def c2(W):
    s = scenes.scene_c2()
    return dict(s=s, geom=W.Geometry.from_scene(s), pts=_t(s.points), u=exact_solution(s, s.points),
                allow=_dirichlet_grad_bound(s, _grad_re_z3))


@pytest.mark.parametrize("wpp", [256, 16384])
def test_c2_full_grid_uniform_per_point_closed_form(W, c2, wpp):
    s = c2["s"]
    say("C2 full grid uniform,", s.n_points, "x", wpp)
    r = _solve(W, c2["geom"], s, c2["pts"], wpp, 18944)
    _check_run(r, s.n_points * wpp)
    # near the holes a few walks per thousand escape to the outer boundary,
    # where |u| is large: the walk values of those points are skewed
    info = zscore_check(r["mean"], r["se"], c2["u"], r["n"], allow=c2["allow"], skewed=True,
                        label="C2 uniform %d wpp" % wpp)
    say("  ", info)


def test_c2_online_guided_per_point_closed_form(W, c2):
    """The path the benchmark times (records, tail pass, Adam, then
    inference-only walks): every point within 3 SE of Re z^3, nothing dropped
    or non-finite, and per point consistent with the uniform estimate."""
    s = c2["s"]
    say("C2 full grid online guided,", s.n_points, "x 256")
    g = _online(W, c2["geom"], s, c2["pts"], 256, 18945, guide_seed=1)
    _check_run(g, s.n_points * 256)
    assert g["info"]["records_dropped"] == 0 and g["info"]["adam_steps"] > 0, g["info"]
    info = zscore_check(g["mean"], g["se"], c2["u"], g["n"], allow=c2["allow"], skewed=True, label="C2 online guided")
    say("  ", info)
    u = _solve(W, c2["geom"], s, c2["pts"], 256, 18944)
    z = two_sample_z(g["mean"], g["se"], u["mean"], u["se"])
    from scipy import stats
    limit = stats.binom.ppf(1 - 1e-6, z.size, 2 * stats.t.sf(3.0, 255))
    say("  guided vs uniform: mean z %.4f, |z| > 3 at %d of %d (limit %d)" % (z.mean(), np.sum(np.abs(z) > 3),
                                                                          z.size, limit))
    assert abs(z.mean()) <= 5.0 / np.sqrt(z.size)
    assert np.sum(np.abs(z) > 3) <= limit


# ----------------------------------------------------------------------------- 3D workloads at full geometric size

def _sample(s, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(s.n_points, n, replace=False))


def test_c4_full_mesh_per_point_closed_form_uniform_and_guided(W):
    """The 215k-triangle mixed problem (u = x^2 - y^2) on 8192 seeded points
    of its z = 0 lattice: uniform at 4096 walks and the online-guided solve at
    256 walks (training through 64), each point against the closed form."""
    s = scenes.scene_c4()
    ids = _sample(s, 8192, 4441)
    pts = _t(s.points[ids])
    u = exact_solution(s, s.points[ids])
    allow = _dirichlet_grad_bound(s, _grad_x2_y2)
    geom = W.Geometry.from_scene(s)
    say("C4 full mesh,", s.prims.shape[0], "triangles, 8192 points")
    a = _solve(W, geom, s, pts, 4096, 18944)
    _check_run(a, 8192 * 4096)
    say("  ", zscore_check(a["mean"], a["se"], u, a["n"], allow=allow, label="C4 uniform"))
    g = _online(W, geom, s, pts, 256, 18945, guide_seed=3)
    _check_run(g, 8192 * 256)
    assert g["info"]["records_dropped"] == 0
    say("  ", zscore_check(g["mean"], g["se"], u, g["n"], allow=allow, label="C4 online guided"))


@pytest.mark.parametrize("case", ["source", "neumann", "mixed"])
def test_c5_full_mesh_manufactured_solutions(W, case):
    """The 1M-triangle mesh of the Poisson workload on 8192 random interior
    points, uniform and online-guided, against closed forms:
    * source: u = |x|^2 (source 6) with every face Dirichlet -- the 3D source
      term at full size, per point;
    * neumann: u = x^2 - y^2 with the Neumann upper half -- the Neumann term
      at full size, per point;
    * mixed: u = |x|^2 (source 6) with the Neumann upper half.  Its Neumann
      data 2 x . n_out are large and one-signed, and for a walker on the
      surface the term G_r(rho) h with area-sampled points has a 1/rho
      singularity whose variance diverges logarithmically: per-point sample
      SEs over 1024 walks are unreliable, so this case is held to the grid
      average (mean deviation within 5 SE plus the epsilon-shell allowance)
      and its per-point figures are reported."""
    s = scenes.scene_c5_manufactured(n_random=8192)
    if case == "source":
        s = dataclasses.replace(s, bc=np.zeros_like(s.bc))
        grad = _grad_r2
    elif case == "neumann":
        s = dataclasses.replace(s, g=scenes._kind("x2_minus_y2"), h=scenes._kind("x2_minus_y2"), f=scenes._zero(),
                                u_exact=scenes._kind("x2_minus_y2"))
        grad = _grad_x2_y2
    else:
        grad = _grad_r2
    pts = _t(s.points)
    u = exact_solution(s, s.points)
    allow = _dirichlet_grad_bound(s, grad)
    geom = W.Geometry.from_scene(s)
    say("C5 mesh", case, s.prims.shape[0], "triangles,", s.n_points, "points")
    a = _solve(W, geom, s, pts, 1024, 18944)
    _check_run(a, s.n_points * 1024)
    # guided weights 1 / (|S| p~) make the walk values more skewed than
    # uniform ones; 1024 walks per point (training through 64) keep the
    # per-point SE reliable
    g = _online(W, geom, s, pts, 1024, 18945, guide_seed=5)
    _check_run(g, s.n_points * 1024)
    for label, r in (("uniform", a), ("online guided", g)):
        if case == "mixed":
            dev = r["mean"] - u
            se_g = np.sqrt(np.sum(r["se"] ** 2)) / s.n_points
            z = dev / r["se"]
            say("   %s: mean deviation %.2e (SE %.2e, allowance %.2e); per point mean z %.3f var z %.3f, |z| > 3 at %d"
                % (label, dev.mean(), se_g, allow, z.mean(), z.var(), np.sum(np.abs(z) > 3)))
            assert abs(dev.mean()) <= 5 * se_g + allow
        else:
            say("  ", zscore_check(r["mean"], r["se"], u, r["n"], allow=allow, skewed=True,
                                   label="C5 mesh %s %s" % (case, label)))


def test_3d_gaussian_source_walk_by_walk(W, O):
    """The Gaussian-bump source of the Poisson workload on a 720-triangle
    Dirichlet sphere: 64 points x 256 walks recomputed by the oracle on the
    same Philox words (the source point y = x + s r nu' and f(y) are then the
    same), walk values within FP32 rounding where the paths agree."""
    s = rounded(scenes.scene_sphere_sources())
    wpp = 256
    geom = W.Geometry.from_scene(s)
    say("3D Gaussian source walk by walk:", s.n_points, "x", wpp)
    g = _solve(W, geom, s, _t(s.points), wpp, 18944, per_walk=True)
    o = O.OracleScene(s).solve(wpp=wpp, per_walk=True)
    same = g["walk_steps"] == o["walk_steps"]
    dv = np.abs(g["walk_value"] - o["walk_value"])[same]
    tol = 1e-4 * np.maximum(1.0, np.abs(o["walk_value"][same]))
    say("  identical step counts %.4f, values within tol %.4f, max |dv| %.2e" % (same.mean(), np.mean(dv <= tol),
                                                                               dv.max()))
    assert same.mean() > 0.99
    assert np.mean(dv <= tol) > 0.995
    mo, so, _ = O.estimates(o)
    z = two_sample_z(g["mean"], g["se"], mo, so)
    assert np.all(np.abs(z) < 1.0), z      # the same walks: far tighter than the sampling error
