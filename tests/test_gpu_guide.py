"""GPU parity of the guide: network inference, MIS direction draws, guided
walks (unbiasedness), training records / tail pass, and the hand-written
backward, all against the FP64 references in ``oracle``."""
import math

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_common import exact_solution, rounded, say
from tests.stats import two_sample_z, zscore_check

pytestmark = pytest.mark.gpu


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


def _ref_cfg(cfg):
    from oracle import guide_ref as G
    d = cfg.dim
    lo = np.asarray(cfg.aabb_lo[:d], np.float32).astype(np.float64)
    hi = np.asarray(cfg.aabb_hi[:d], np.float32).astype(np.float64)
    return G.GuideConfig(dim=d, levels=cfg.levels, feats=cfg.feats, log2_T=cfg.log2_table, n_min=cfg.n_min,
                         n_max=cfg.n_max, hidden=cfg.hidden, n_hidden=cfg.n_hidden, K=cfg.K, aabb_lo=lo, aabb_hi=hi)


def _random_params(rcfg, rng, grid_scale=0.5, mlp_gain=1.0):
    p = [rng.uniform(-grid_scale, grid_scale, rcfg.n_grid_params)]
    for a, b in rcfg.layer_shapes():
        p.append(rng.uniform(-1, 1, a * b) * math.sqrt(6 / a) * mlp_gain)
    return np.concatenate(p)


def _half(p):
    return np.asarray(p, np.float32).astype(np.float16).astype(np.float64)


def _guide_setup(W, scene, seed=0, mlp_gain=1.0, **kw):
    cfg = W.GuideConfig.for_scene(scene, **kw)
    g = W.Guide(cfg, seed=seed + 1)
    rcfg = _ref_cfg(cfg)
    rng = np.random.default_rng(100 + seed)
    params = _random_params(rcfg, rng, mlp_gain=mlp_gain)
    g.set_params(params)
    torch.cuda.synchronize()
    return g, cfg, rcfg, _half(params)


def _scene_2d():
    return rounded(scenes.scene_c2())


def _scene_3d():
    P, T = scenes.geodesic_sphere(8)
    cen = P[T].mean(1)
    bc = (cen[:, 2] > 0).astype(np.uint8)
    rng = np.random.default_rng(4)
    Q = rng.normal(size=(400, 3))
    Q = Q / np.linalg.norm(Q, axis=1, keepdims=True) * rng.uniform(0, 0.9, (400, 1))
    s = scenes.Scene("sphere8", 3, P, T, bc, Q, g=(4, np.zeros(0)), h=(4, np.zeros(0)), f=(0, np.zeros(0)),
                     u_exact=(4, np.zeros(0)), eps=1e-3, max_steps=4096, rr_start=128, rr_q=0.99)
    return rounded(s)


# ----------------------------------------------------------------------------- inference

@pytest.mark.parametrize("dim,K", [(2, 8), (3, 8), (2, 4), (2, 16)])
def test_guide_infer_matches_fp64_reference(W, dim, K):
    from oracle import guide_ref as G
    s = _scene_2d() if dim == 2 else _scene_3d()
    kw = dict(K=K) if dim == 2 else dict(log2_table=14, K=K)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=dim, **kw)
    rng = np.random.default_rng(7)
    lo, hi = rcfg.lo, rcfg.hi
    pts = np.asarray(rng.uniform(lo - 0.05, hi + 0.05, (4096, dim)), np.float32).astype(np.float64)
    say("guide infer", dim, cfg)
    y = g.infer(_t(pts)).double().cpu().numpy()
    with torch.no_grad():
        y_mixed = G.forward(rcfg, p16, pts, round_inputs=True).numpy()
        y_exact = G.forward(rcfg, p16, pts).numpy()
    scale = np.sqrt(np.mean(y_mixed ** 2))
    err = np.abs(y - y_mixed) / scale
    say("infer err vs mixed-precision ref: max %.2e p99 %.2e; vs exact-arith ref max %.2e"
        % (err.max(), np.percentile(err, 99), (np.abs(y - y_exact) / scale).max()))
    assert np.percentile(err, 99.9) < 2e-3 and err.max() < 2e-2
    assert (np.abs(y - y_exact) / scale).max() < 5e-2


# ----------------------------------------------------------------------------- sampler

def _philox_blocks(O, n, j, step, blocks, seed):
    ctr = np.zeros((n * len(blocks), 4), np.uint32)
    ctr[:, 0] = np.repeat(np.arange(n), len(blocks))
    ctr[:, 1] = j
    ctr[:, 2] = step
    ctr[:, 3] = np.tile(blocks, n)
    w = O.philox_batch(ctr, [seed & 0xFFFFFFFF, seed >> 32]).reshape(n, len(blocks), 4)
    return (w >> 8).astype(np.float64) * 2.0 ** -24


@pytest.mark.parametrize("dim,mode,K,reflected",
                         [(d, m, 8, True) for d in (2, 3) for m in ("mis_learned", "mis_fixed", "guided_only")]
                         + [(2, "mis_learned", 4, True), (2, "mis_learned", 16, True)]
                         + [(2, "mis_learned", 8, False), (3, "mis_learned", 8, False), (2, "guided_only", 8, False)])
def test_guide_sample_matches_reference_on_same_words(W, O, dim, mode, K, reflected):
    from oracle import guide_ref as G
    s = _scene_2d() if dim == 2 else _scene_3d()
    kw = dict(K=K) if dim == 2 else dict(log2_table=14, K=K)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=10 + dim, **kw)
    g.reflect = reflected
    assert g.reflect == reflected
    rng = np.random.default_rng(8 + dim)
    n = 2048
    pts = np.asarray(rng.uniform(rcfg.lo, rcfg.hi, (n, dim)), np.float32).astype(np.float64)
    nrm = rng.normal(size=(n, dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    nrm[: n // 2] = 0.0                                  # first half interior, second half on a wall
    nrm = np.asarray(nrm, np.float32).astype(np.float64)
    seed, j = 1234567, 5
    say("guide sample", dim, mode, "reflected" if reflected else "not reflected")
    nu, pdf = g.sample(_t(pts), _t(nrm), sampling=mode, c_fixed=0.35, seed=seed, walk_index=j)
    y = g.infer(_t(pts)).double().cpu().numpy()
    nu = nu.double().cpu().numpy()
    pdf = pdf.double().cpu().numpy()
    mu, kappa, lam, c = G.map_outputs(y, dim, cfg.K)
    if mode == "mis_fixed":
        c = np.full(n, 0.35)
    elif mode == "guided_only":
        c = np.ones(n)
    words = _philox_blocks(O, n, j, 0, list(range(0, 4)) + list(range(4, 4 + 16)), seed)
    agree = 0
    wasted = 0
    pdf_err = []
    for i in range(n):
        onN = bool(np.any(nrm[i] != 0))
        b0 = words[i, 0]
        b3 = words[i, 3]
        bf = [tuple(words[i, 4 + t, :3]) for t in range(16)]
        nu_r, p_r, _ = G.sample_direction(dim, mu[i], kappa[i], lam[i], c[i], b0, b3, bf, onN, nrm[i] if onN else None,
                                          reflected)
        agree += np.linalg.norm(nu_r - nu[i]) < 2e-3 and (pdf[i] < 0) == (p_r == 0.0)
        if pdf[i] < 0:
            # a wasted draw: only without reflection, only into the wall
            assert onN and not reflected and np.dot(nu[i], nrm[i]) <= 1e-6
            wasted += 1
            continue
        # pdf of the GPU's own direction under the same mapped parameters
        p_at = G.mis_pdf(nu[i], mu[i], kappa[i], lam[i], c[i], dim, onN, nrm[i] if onN else None, reflected)
        pdf_err.append(abs(pdf[i] - p_at) / p_at)
        if onN:
            assert np.dot(nu[i], nrm[i]) >= -1e-6
    pdf_err = np.asarray(pdf_err)
    say("sample agree %.4f, wasted %d, pdf rel err p99 %.2e max %.2e"
        % (agree / n, wasted, np.percentile(pdf_err, 99), pdf_err.max()))
    assert agree / n > 0.99
    assert (wasted > 0) == (not reflected)
    assert np.percentile(pdf_err, 99) < 1e-4 and pdf_err.max() < 1e-2
    np.testing.assert_allclose(np.linalg.norm(nu, axis=1), 1.0, atol=1e-5)


# ----------------------------------------------------------------------------- guided walks

def _solve(W, s, geom, pb, pts, wpp, guide=None, seed=18944, per_walk=False, records=None):
    n = pts.shape[0]
    wv = torch.empty(n * wpp, dtype=torch.float32, device="cuda") if (per_walk or records is not None) else None
    ws = torch.empty(n * wpp, dtype=torch.int32, device="cuda") if per_walk else None
    acc = W.solve(geom, pb, _t(pts), wpp, seed=seed, guide=guide, walk_value=wv, walk_steps=ws, records=records)
    torch.cuda.synchronize()
    m, se, cnt = acc.estimates()
    out = dict(mean=m.cpu().numpy(), se=se.cpu().numpy(), n=cnt.cpu().numpy(), stats=acc.stats(), wv=wv)
    if per_walk:
        out.update(walk_value=wv.double().cpu().numpy(), walk_steps=ws.cpu().numpy())
    return out


def test_c_zero_reproduces_uniform_trajectories(W):
    s = _scene_2d()
    pts = s.points[::97][:256]
    geom = W.Geometry.from_scene(s)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=21)
    say("c=0 vs uniform")
    u = _solve(W, s, geom, W.Problem.from_scene(s), pts, 32, per_walk=True)
    c0 = _solve(W, s, geom, W.Problem.from_scene(s, sampling="mis_fixed", c_fixed=0.0), pts, 32, guide=g,
                per_walk=True)
    np.testing.assert_array_equal(u["walk_steps"], c0["walk_steps"])
    np.testing.assert_allclose(c0["walk_value"], u["walk_value"], rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("mode", ["mis_learned", "guided_only"])
def test_guided_c1_unbiased(W, mode):
    s = rounded(scenes.scene_c1())
    geom = W.Geometry.from_scene(s)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=31)
    say("guided C1", mode)
    r = _solve(W, s, geom, W.Problem.from_scene(s, sampling=mode), s.points, 1024, guide=g)
    zscore_check(r["mean"], r["se"], exact_solution(s, s.points), r["n"], label="guided C1 " + mode)
    assert r["stats"]["nonfinite"] == 0


def test_guided_c2_unbiased_with_reflection(W):
    """Neumann boundary: reflected mixture + MIS must stay unbiased."""
    s = _scene_2d()
    pts = s.points[::11]
    geom = W.Geometry.from_scene(s)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=41)
    say("guided C2", len(pts))
    # the problem's reflection flag must match the guide's setting
    with pytest.raises(RuntimeError, match="reflect"):
        _solve(W, s, geom, W.Problem.from_scene(s, sampling="mis_learned", reflect=False), pts[:8], 4, guide=g)
    r = _solve(W, s, geom, W.Problem.from_scene(s, sampling="mis_learned"), pts, 512, guide=g)
    zscore_check(r["mean"], r["se"], exact_solution(s, pts), r["n"], label="guided C2")
    u = _solve(W, s, geom, W.Problem.from_scene(s), pts, 512)
    z = two_sample_z(r["mean"], r["se"], u["mean"], u["se"])
    assert abs(z.mean()) < 5 / np.sqrt(len(z)) and np.mean(np.abs(z) > 3) < 0.01


def test_guided_c2_unbiased_without_reflection(W):
    """Reflection off (the ablation of the reflection step): guided draws into
    the wall end the walk with a zero recursive term, and the estimate must
    stay unbiased; records are written only for directions actually used."""
    s = _scene_2d()
    pts = s.points[::11]
    geom = W.Geometry.from_scene(s)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=42)
    g.reflect = False
    say("guided C2 without reflection", len(pts))
    with pytest.raises(RuntimeError, match="reflect"):
        _solve(W, s, geom, W.Problem.from_scene(s, sampling="mis_learned"), pts[:8], 4, guide=g)
    pb = W.Problem.from_scene(s, sampling="mis_learned", reflect=False)
    r = _solve(W, s, geom, pb, pts, 512, guide=g)
    zscore_check(r["mean"], r["se"], exact_solution(s, pts), r["n"], label="guided C2 no reflection")
    assert r["stats"]["nonfinite"] == 0
    rec = W.Records(2, capacity=256 * 16 * 256)
    r = _solve(W, s, geom, pb, pts[:256], 16, guide=g, records=rec)
    nrec = rec.n()
    assert nrec == r["stats"]["records"] and r["stats"]["records_dropped"] == 0
    F = {k: v.cpu().numpy() for k, v in rec.fields(nrec).items()}
    on = np.any(F["n"] != 0, axis=1)
    assert on.any()
    # every recorded direction at a Neumann point lies in the valid half
    assert np.all(np.sum(F["nu"][on] * F["n"][on], axis=1) >= -1e-6)
    assert np.all(F["p_sample"] > 0)


def test_guided_3d_sphere_unbiased(W):
    s = _scene_3d()
    geom = W.Geometry.from_scene(s)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=51, log2_table=14)
    say("guided 3D sphere")
    r = _solve(W, s, geom, W.Problem.from_scene(s, sampling="mis_learned"), s.points, 1024, guide=g)
    zscore_check(r["mean"], r["se"], exact_solution(s, s.points), r["n"], label="guided 3D")


# ----------------------------------------------------------------------------- records + tail pass

def test_records_and_tail_pass_match_reverse_recursion(W, O):
    """C1 Poisson (source term, no Neumann term): with c = 0 the GPU walks follow
    the oracle's trajectories; every record's training target |V_{k+1}| must
    match the oracle's reverse recursion V_k = c_k + w_k V_{k+1}."""
    from oracle.guide_ref import tail_targets
    s = rounded(scenes.scene_c1_poisson())
    pts = s.points[::13]
    n, wpp = pts.shape[0], 8
    geom = W.Geometry.from_scene(s)
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=61)
    rec = W.Records(2, capacity=n * wpp * 64)
    say("records / tail pass")
    r = _solve(W, s, geom, W.Problem.from_scene(s, sampling="mis_fixed", c_fixed=0.0), pts, wpp, guide=g,
               per_walk=True, records=rec)
    W.tail_pass(rec, r["wv"])
    torch.cuda.synchronize()
    nrec = rec.n()
    assert nrec == r["stats"]["records"] and r["stats"]["records_dropped"] == 0
    F = {k: v.cpu().numpy() for k, v in rec.fields(nrec).items()}
    # records of one walk are appended in step order
    order = np.argsort(F["slot"], kind="stable")
    slots = F["slot"][order]
    pt = F["p_t"][order]
    o = O.OracleScene(s)
    checked = 0
    starts = np.searchsorted(slots, np.arange(n * wpp))
    ends = np.searchsorted(slots, np.arange(n * wpp), side="right")
    for w in range(0, n * wpp, 7):
        p, j = divmod(w, wpp)
        tr = o.walk_trace(pts[p], p, j)
        if len(tr["c"]) != ends[w] - starts[w]:
            continue      # an FP32/FP64 branch flip changed this trajectory
        V0, tails = tail_targets(tr["c"], tr["w"], tr["terminal"], killed=tr["status"] == 2)
        np.testing.assert_allclose(pt[starts[w]:ends[w]], tails, rtol=2e-4, atol=2e-5)
        assert abs(V0 - r["walk_value"][w]) < 1e-4 * max(1, abs(V0))
        checked += 1
    assert checked > 0.9 * len(range(0, n * wpp, 7))


# ----------------------------------------------------------------------------- loss + backward

def _synthetic_records(W, rcfg, n, rng, dim):
    rec = W.Records(dim, capacity=n)
    x = np.asarray(rng.uniform(rcfg.lo, rcfg.hi, (n, dim)), np.float32)
    nu = rng.normal(size=(n, dim))
    nu /= np.linalg.norm(nu, axis=1, keepdims=True)
    on = rng.random(n) < 0.4
    nr = rng.normal(size=(n, dim))
    nr /= np.linalg.norm(nr, axis=1, keepdims=True)
    flip = (np.sum(nu * nr, 1) < 0) & on
    nu[flip] -= 2 * np.sum(nu[flip] * nr[flip], 1, keepdims=True) * nr[flip]
    nr[~on] = 0
    nu = np.asarray(nu, np.float32)
    nr = np.asarray(nr, np.float32)
    ps = np.asarray(rng.uniform(0.05, 0.5, n), np.float32)
    pt = np.asarray(np.abs(rng.normal(size=n)), np.float32)
    D = np.zeros((3 * dim + 5, n), np.float32)
    D[0:dim] = x.T
    D[dim:2 * dim] = nu.T
    D[2 * dim:3 * dim] = nr.T
    D[3 * dim] = ps
    D[3 * dim + 4] = pt
    rec.data.copy_(torch.as_tensor(D))
    rec.count.fill_(n)
    f64 = lambda a: np.asarray(a, np.float64)  # noqa: E731
    return rec, (f64(x), f64(nu), f64(nr), on, f64(ps), f64(pt))


@pytest.mark.parametrize("dim,K,reflected", [(2, 8, True), (3, 8, True), (2, 4, True), (2, 16, True),
                                             (2, 8, False), (3, 8, False)])
def test_loss_and_backward_match_fp64_reference(W, dim, K, reflected):
    from oracle import guide_ref as G
    s = _scene_2d() if dim == 2 else _scene_3d()
    kw = dict(K=K) if dim == 2 else dict(log2_table=14, K=K)
    # MLP weights at 0.6x He scale keep kappa' in the range a trained guide uses
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=70 + dim, mlp_gain=0.6, **kw)
    g.reflect = reflected
    rng = np.random.default_rng(71 + dim)
    n = 3000
    rec, batch = _synthetic_records(W, rcfg, n, rng, dim)
    say("loss/backward", dim)
    loss = g.loss_fwd(rec).double().cpu().numpy()
    with torch.no_grad():
        y = G.forward(rcfg, p16, batch[0], round_inputs=True)
        ref_loss = G.loss_per_sample(rcfg, y, *batch[1:], reflected=reflected).numpy()
    # Both networks round every layer input to FP16.  Where a value lies
    # within FP32 rounding of an FP16 rounding boundary, the GPU (FP32
    # accumulation) and the reference (FP64) may round it to different
    # neighbours, both correct; such a record's outputs then differ by up to
    # about one FP16 step of an input (~1e-3 of the output scale), and its
    # loss gradient, steep in the mean directions of a fresh network, by more.
    # Every record is held to that bound; the records where the two forward
    # passes agree to FP32 rounding (98-99% of them) are compared tightly.
    y_gpu = g.infer(_t(batch[0])).double().cpu().numpy()
    yscale = np.sqrt(np.mean(y.numpy() ** 2))
    yerr = np.abs(y_gpu - y.numpy()).max(1) / yscale
    same = yerr < 1e-5
    say("forward: %d of %d records agree to FP32 rounding, max err elsewhere %.2e"
        % (same.sum(), n, yerr.max()))
    assert yerr.max() < 2e-3 and same.mean() > 0.97
    lerr = np.abs(loss - ref_loss) / (np.abs(ref_loss) + np.mean(np.abs(ref_loss)))
    say("loss rel err max %.2e (records with equal rounding: %.2e)" % (lerr.max(), lerr[same].max()))
    assert lerr.max() < 2e-3 and lerr[same].max() < 1e-5
    # gradient of the loss over those records via the autograd Function
    mask = torch.as_tensor(same, dtype=torch.float32, device="cuda")
    params = g.master.clone().requires_grad_(True)
    lv = W.GuideLoss.apply(params, g, rec, 0, n, 0.2)
    ((lv * mask).sum() / n).backward()
    grad = params.grad.double().cpu().numpy()
    # FP64 reference gradient of the same loss through the reference's own
    # forward pass (FP16-rounded layer inputs); no GPU value enters it
    p = torch.tensor(p16, dtype=torch.float64, requires_grad=True)
    y_ref = G.forward(rcfg, p, batch[0], round_inputs=True)
    lref = G.loss_per_sample(rcfg, y_ref, *batch[1:], reflected=reflected)
    ((lref * torch.as_tensor(same, dtype=torch.float64)).sum() / n).backward()
    ref_grad = p.grad.numpy()
    rel = np.linalg.norm(grad - ref_grad) / np.linalg.norm(ref_grad)
    ng = rcfg.n_grid_params
    rel_mlp = np.linalg.norm(grad[ng:] - ref_grad[ng:]) / np.linalg.norm(ref_grad[ng:])
    rel_grid = np.linalg.norm(grad[:ng] - ref_grad[:ng]) / np.linalg.norm(ref_grad[:ng])
    say("grad rel err: all %.2e mlp %.2e grid %.2e" % (rel, rel_mlp, rel_grid))
    assert rel < 1e-3 and rel_mlp < 1e-3 and rel_grid < 1e-3
    # level by level: the coarse dense levels are accumulated through LDS, the
    # finer ones by direct atomics, and each must hold on its own
    per = rcfg.T * rcfg.F
    lvl = [np.linalg.norm(grad[l * per:(l + 1) * per] - ref_grad[l * per:(l + 1) * per])
           / np.linalg.norm(ref_grad[l * per:(l + 1) * per]) for l in range(rcfg.L)]
    say("grid rel err per level: " + " ".join("%.1e" % e for e in lvl))
    assert max(lvl) < 1e-3


def test_train_step_fits_known_target(W):
    """Records with nu uniform and p_t a fixed vMF (kappa = 20) at 16 fixed
    positions, 4096 records each: Adam on the guide must drive the loss down to
    near its floor, raise the selection probability c, and put the mixture's
    mass on the target direction.  The floor is (1 + e) times the target's
    entropy, since the expected loss is a cross-entropy against a normalised
    guide; a loss well below it would mean an unnormalised pdf (or records
    memorised per position, which 4096 records per position rule out)."""
    from oracle import guide_ref as G
    s = _scene_2d()
    cfg = W.GuideConfig.for_scene(s)
    g = W.Guide(cfg, seed=81)          # library initialisation: grid U(+-1e-4), MLP He-uniform
    rcfg = _ref_cfg(cfg)
    rng = np.random.default_rng(82)
    n = 1 << 16
    n_pos = 16
    rec = W.Records(2, capacity=n)
    pos = rng.uniform(rcfg.lo + 0.1, rcfg.hi - 0.1, (n_pos, 2))
    x = np.repeat(pos, n // n_pos, axis=0)
    th = rng.uniform(0, 2 * np.pi, n)
    nu = np.stack([np.cos(th), np.sin(th)], 1)
    kt = 20.0
    mu_t = np.array([math.cos(0.7), math.sin(0.7)])
    pt = np.exp(G.vmf_logpdf(nu, mu_t, kt))
    D = np.zeros((11, n), np.float32)
    D[0:2] = x.T
    D[2:4] = nu.T
    D[6] = 1 / (2 * np.pi)
    D[10] = pt
    rec.data.copy_(torch.as_tensor(D))
    rec.count.fill_(n)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for it in range(400):
        g.train_step(rec, 0, n, lr=1e-2, loss_out=loss)
        if it % 50 == 0 or it == 399:
            losses.append(float(loss.item()))
    # entropy of the 2D vMF: log(2 pi I0e(k)) + k (1 - I1/I0)
    from scipy.special import i0e, i1e
    H = math.log(2 * math.pi * i0e(kt)) + kt * (1.0 - i1e(kt) / i0e(kt))
    floor = 1.2 * H
    say("known-target losses", losses, "floor %.4f" % floor)
    assert losses[-1] < losses[0] - 0.5
    assert floor - 0.05 < losses[-1] < floor + 0.15, (losses[-1], floor)
    y = g.infer(_t(pos)).double().cpu().numpy()
    mu, kappa, lam, c = G.map_outputs(y, 2, cfg.K)
    assert np.median(c) > 0.7, c
    # the fitted mixture puts its mass near the target mean at every position
    peak = math.exp(G.vmf_logpdf(mu_t[None], mu_t, kt)[0])
    dens = np.array([G.mixture_pdf(mu_t[None], mu[i], kappa[i], lam[i])[0] for i in range(n_pos)])
    say("density at target mean / target peak", np.round(dens / peak, 3))
    assert np.all(dens > 0.5 * peak), dens / peak


def test_records_sample_draws_rows_uniformly(W):
    """wost_records_sample: every drawn row is a whole row of the source
    (all fields of one record), rows are drawn uniformly over the source's
    written rows, the destination count is m, and an empty source yields an
    empty training set."""
    from paper_2410_18944_amd.guide import sample_records
    from scipy import stats
    n_src, cap, m = 5000, 6000, 1 << 20
    src = W.Records(3, capacity=cap)
    D = np.zeros((14, cap), np.float32)
    D[:, :n_src] = np.arange(n_src, dtype=np.float32)[None, :] + np.arange(14, dtype=np.float32)[:, None] * 1e5
    src.data.copy_(torch.as_tensor(D))
    src.count.fill_(n_src)
    dst = W.Records(3, capacity=m)
    sample_records(src, 77, m, dst)
    torch.cuda.synchronize()
    assert int(dst.count.item()) == m
    out = dst.data.cpu().numpy()
    row = out[0].astype(np.int64)
    assert row.min() >= 0 and row.max() < n_src
    np.testing.assert_array_equal(out, row[None, :].astype(np.float32) + np.arange(14, dtype=np.float32)[:, None] * 1e5)
    cnt = np.bincount(row, minlength=n_src)
    chi2 = np.sum((cnt - m / n_src) ** 2 / (m / n_src))
    assert stats.chi2.sf(chi2, n_src - 1) > 1e-6, chi2
    # another seed draws another sample; an empty source gives count 0
    dst2 = W.Records(3, capacity=m)
    sample_records(src, 78, m, dst2)
    src.count.zero_()
    dst3 = W.Records(3, capacity=16)
    sample_records(src, 79, 16, dst3)
    torch.cuda.synchronize()
    assert not torch.equal(dst.data, dst2.data)
    assert int(dst3.count.item()) == 0
