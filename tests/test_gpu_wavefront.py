"""The multi-kernel wavefront solver (wost_solve_wavefront) against the
persistent kernel walk by walk, and against the FP64 oracle and closed forms.
Both solvers give a walk the same random words and run the same traversal
code, so per-walk step counts and values must agree."""
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


def _run(W, s, pts, wpp, engine, guide=None, records=None, seed=18944, **pkw):
    geom = W.Geometry.from_scene(s)
    pb = W.Problem.from_scene(s, **pkw)
    n = pts.shape[0]
    wv = torch.empty(n * wpp, dtype=torch.float32, device="cuda")
    ws = torch.empty(n * wpp, dtype=torch.int32, device="cuda")
    acc = W.solve(geom, pb, _t(pts), wpp, seed=seed, guide=guide, walk_value=wv, walk_steps=ws, records=records,
                  engine=engine)
    torch.cuda.synchronize()
    m, se, cnt = acc.estimates()
    return dict(mean=m.cpu().numpy(), se=se.cpu().numpy(), n=cnt.cpu().numpy(), stats=acc.stats(),
                walk_value=wv.double().cpu().numpy(), walk_steps=ws.cpu().numpy())


def _same_walks(a, b, label):
    same = a["walk_steps"] == b["walk_steps"]
    dv = np.abs(a["walk_value"] - b["walk_value"])
    tol = 1e-5 * np.maximum(1.0, np.abs(b["walk_value"]))
    say("%s: identical step counts %.6f, max |dv| %.2e" % (label, same.mean(), dv[same].max() if same.any() else 0))
    assert same.mean() > 0.999, same.mean()
    assert np.all(dv[same] <= tol[same])
    for k in ("walks", "steps", "truncated", "rr_killed", "nonfinite"):
        assert abs(a["stats"][k] - b["stats"][k]) <= 1e-3 * max(1, b["stats"][k]), (k, a["stats"][k], b["stats"][k])


def _scene(name):
    if name == "C1":
        return rounded(scenes.scene_c1())
    if name == "C1 Poisson":
        return rounded(scenes.scene_c1_poisson())
    if name == "C2":
        return rounded(scenes.scene_c2())
    if name == "halfdisk":
        return rounded(scenes.scene_halfdisk_neumann())
    return rounded(scenes.scene_cube_box())


@pytest.mark.parametrize("name", ["C1", "C1 Poisson", "C2", "halfdisk", "cube"])
def test_wavefront_matches_persistent_walk_by_walk(W, name):
    s = _scene(name)
    pts = s.points if s.n_points <= 2048 else s.points[::23]
    wpp = 16
    say("wavefront vs persistent, uniform", name, len(pts), "x", wpp)
    a = _run(W, s, pts, wpp, "wavefront")
    b = _run(W, s, pts, wpp, "persistent")
    _same_walks(a, b, name)
    assert a["stats"]["walks"] == len(pts) * wpp
    assert a["stats"]["steps"] == int(a["walk_steps"].sum())


@pytest.mark.parametrize("reflect,streams", [(True, 1), (False, 1), (True, 2)])
def test_wavefront_guided_matches_persistent_with_records(W, reflect, streams):
    from tests.test_gpu_guide import _guide_setup
    from paper_2410_18944_amd import api
    api.set_wavefront_streams(streams)
    s = rounded(scenes.scene_c2())
    pts = s.points[::41]
    wpp = 8
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=81)
    g.reflect = reflect
    say("wavefront vs persistent, guided", len(pts), "x", wpp, "reflect", reflect, "streams", streams)
    recs = {}
    out = {}
    for eng in ("wavefront", "persistent"):
        rec = W.Records(2, capacity=len(pts) * wpp * 256)
        out[eng] = _run(W, s, pts, wpp, eng, guide=g, records=rec, sampling="mis_learned", reflect=reflect)
        n = rec.n()
        assert n == out[eng]["stats"]["records"] and out[eng]["stats"]["records_dropped"] == 0
        F = {k: v.cpu().numpy() for k, v in rec.fields(n).items()}
        # rows of one walk are appended in step order by both solvers; the
        # interleaving of walks differs
        order = np.argsort(F["slot"], kind="stable")
        recs[eng] = {k: v[order] for k, v in F.items()}
    _same_walks(out["wavefront"], out["persistent"], "guided")
    a, b = recs["wavefront"], recs["persistent"]
    assert len(a["slot"]) == len(b["slot"])
    np.testing.assert_array_equal(a["slot"], b["slot"])
    for k in ("x", "nu", "n", "p_sample", "prefix", "t_next"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-5, atol=1e-6, err_msg=k)
    api.set_wavefront_streams(1)


def test_wavefront_3d_guided_matches_persistent(W):
    from tests.test_gpu_guide import _guide_setup, _scene_3d
    from paper_2410_18944_amd import api
    s = _scene_3d()
    g, cfg, rcfg, p16 = _guide_setup(W, s, seed=82, log2_table=14)
    say("wavefront vs persistent, guided 3D, two streams")
    api.set_wavefront_streams(2)
    try:
        a = _run(W, s, s.points, 16, "wavefront", guide=g, sampling="mis_learned")
    finally:
        api.set_wavefront_streams(1)
    b = _run(W, s, s.points, 16, "persistent", guide=g, sampling="mis_learned")
    _same_walks(a, b, "guided 3D")


def test_wavefront_c2_against_oracle_and_closed_form(W, O):
    s = rounded(scenes.scene_c2())
    idx = np.arange(0, s.n_points, 173)[:192]
    pts = s.points[idx]
    say("wavefront C2 vs oracle", len(pts))
    o = O.OracleScene(s).solve(points=pts, wpp=64, per_walk=True)
    g = _run(W, s, pts, 64, "wavefront")
    same = g["walk_steps"] == o["walk_steps"]
    assert same.mean() > 0.97, same.mean()
    mo, so, no = O.estimates(o)
    z = two_sample_z(g["mean"], g["se"], mo, so)
    assert np.mean(np.abs(z) > 3) < 0.02 and abs(z.mean()) < 5 / np.sqrt(len(z))
    c1 = rounded(scenes.scene_c1())
    r = _run(W, c1, c1.points, 1024, "wavefront")
    zscore_check(r["mean"], r["se"], exact_solution(c1, c1.points), r["n"], label="wavefront C1")


def test_wavefront_edge_cases(W):
    s = rounded(scenes.scene_c1())
    say("wavefront edge cases")
    one = _run(W, s, s.points[:1], 1, "wavefront")
    ref = _run(W, s, s.points[:1], 1, "persistent")
    np.testing.assert_array_equal(one["walk_steps"], ref["walk_steps"])
    # a ragged count of walks (not a multiple of the wave width)
    a = _run(W, s, s.points[:37], 3, "wavefront")
    b = _run(W, s, s.points[:37], 3, "persistent")
    _same_walks(a, b, "ragged")
    # step cap 0: every walk ends at its first closest-point query
    c = _run(W, s, s.points[:64], 4, "wavefront", max_steps=0)
    d = _run(W, s, s.points[:64], 4, "persistent", max_steps=0)
    assert np.all(c["walk_steps"] == 1)
    _same_walks(c, d, "max_steps 0")
    from paper_2410_18944_amd import api
    # traversal-cost counters are kept by the persistent kernel only
    from paper_2410_18944_amd import api
    cost = torch.zeros(18, dtype=torch.int64, device="cuda")
    api.set_cost_counters(cost)
    try:
        with pytest.raises(RuntimeError, match="cost"):
            _run(W, s, s.points[:8], 2, "wavefront")
    finally:
        api.set_cost_counters(None)
