"""The GPU-built linear BVH (wost_lbvh_build / wost_lbvh_closest): closest
distances against the host-built hierarchy of the same primitives and
against the FP64 oracle's brute force, and the structure of the built
hierarchy checked on the host (every primitive in exactly one leaf, every
box containing what lies below it)."""
import numpy as np
import pytest
import torch

import scenes
from tests.gpu_common import rounded, say

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


def _records(dim, verts, prims):
    """float4 records: 2D (ax, ay, bx, by); 3D (a, b, c) in three float4."""
    v = np.asarray(verts, np.float32)
    if dim == 2:
        return np.concatenate([v[prims[:, 0]], v[prims[:, 1]]], 1).astype(np.float32)
    t = np.concatenate([v[prims[:, 0]], v[prims[:, 1]], v[prims[:, 2]], np.zeros((len(prims), 3), np.float32)], 1)
    return t.astype(np.float32)


def _check_structure(bv, dim, recs, leaf_size):
    """Walk the four-wide tree on the host."""
    stride = 2 * dim + 1
    nodes = bv.nodes.cpu().numpy().reshape(-1, stride, 4)[: bv.n_nodes]
    orig = bv.orig.cpu().numpy()
    n = bv.n
    assert np.array_equal(np.sort(orig), np.arange(n))
    per = 1 if dim == 2 else 3
    sp = bv.prims.cpu().numpy().reshape(n, per * 4)
    np.testing.assert_array_equal(sp, recs.reshape(n, -1)[orig])
    if dim == 2:
        pts = sp.reshape(n, 2, 2)
    else:
        pts = sp[:, :9].reshape(n, 3, 3)
    plo, phi = pts.min(1), pts.max(1)
    seen = np.zeros(n, np.int64)
    visited = np.zeros(bv.n_nodes, np.int64)
    depth = 0
    stack = [(0, 1)]
    while stack:
        k, dep = stack.pop()
        depth = max(depth, dep)
        visited[k] += 1
        refs = nodes[k, 2 * dim].view(np.int32)
        for c in range(4):
            r = int(refs[c])
            lo = np.array([nodes[k, a, c] for a in range(dim)])
            hi = np.array([nodes[k, dim + a, c] for a in range(dim)])
            if r == np.iinfo(np.int32).min:
                assert np.all(lo == np.inf) and np.all(hi == -np.inf)
                continue
            if r < 0:
                first, count = (-1 - r) // 64, (-1 - r) % 64 + 1
                assert count <= max(leaf_size, 1)
                seen[first:first + count] += 1
                assert np.all(plo[first:first + count] >= lo) and np.all(phi[first:first + count] <= hi)
            else:
                assert 0 < r < bv.n_nodes
                clo = np.array([nodes[r, a][np.isfinite(nodes[r, a])].min() if np.isfinite(nodes[r, a]).any() else np.inf
                                for a in range(dim)])
                chi = np.array([nodes[r, dim + a][np.isfinite(nodes[r, dim + a])].max()
                                if np.isfinite(nodes[r, dim + a]).any() else -np.inf for a in range(dim)])
                assert np.all(clo >= lo) and np.all(chi <= hi)
                stack.append((r, dep + 1))
    assert np.all(seen == 1), (seen.min(), seen.max())
    assert np.all(visited == 1)
    assert depth == bv.levels


def _dirichlet(s):
    return s.prims[s.bc == 0]


@pytest.mark.parametrize("name", ["C2", "C4", "C5"])
def test_lbvh_closest_matches_host_hierarchy_and_oracle(W, O, name):
    from paper_2410_18944_amd.api import Lbvh
    s = rounded({"C2": scenes.scene_c2, "C4": scenes.scene_c4, "C5": scenes.scene_c5}[name]())
    dp = _dirichlet(s)
    recs = _records(s.dim, s.verts, dp)
    say("LBVH", name, len(dp), "primitives")
    bv = Lbvh(s.dim, torch.as_tensor(recs, device="cuda").reshape(-1), leaf_size=4)
    torch.cuda.synchronize()
    say("nodes %d levels %d" % (bv.n_nodes, bv.levels))
    if len(dp) <= 50000:
        _check_structure(bv, s.dim, recs, 4)
    rng = np.random.default_rng(31)
    pts = s.points[rng.choice(s.n_points, min(s.n_points, 20000), replace=False)]
    # points off the query grid too: near and beyond the boundary
    lo, hi = s.verts.min(0), s.verts.max(0)
    extra = rng.uniform(lo - 0.2 * (hi - lo), hi + 0.2 * (hi - lo), (5000, s.dim))
    pts = np.asarray(np.concatenate([pts, extra]), np.float32).astype(np.float64)
    tp = torch.as_tensor(pts, dtype=torch.float32, device="cuda")
    d_l, p_l = bv.closest(tp)
    # the host-built hierarchy over the same primitives
    sd = W.Geometry(s.dim, s.verts, dp, np.zeros(len(dp), np.uint8))
    q = sd.query(tp, silhouette=False)
    torch.cuda.synchronize()
    d_l, p_l = d_l.double().cpu().numpy(), p_l.cpu().numpy()
    d_h = q["d_dir"].double().cpu().numpy()
    L = float(np.linalg.norm(hi - lo))
    err = np.abs(d_l - d_h)
    say("max |d_lbvh - d_host| %.3e" % err.max())
    assert np.all(err <= 1e-6 * d_h + 1e-7 * L)
    assert np.all((p_l >= 0) & (p_l < len(dp)))
    # the returned primitive is at the returned distance
    # (FP64 distance to that primitive, from the oracle's own routine)
    o = O.OracleScene(s)
    sub = rng.choice(len(pts), 64, replace=False)
    d_o, _ = o.closest_dirichlet(pts[sub])
    assert np.all(np.abs(d_l[sub] - d_o) <= 1e-5 * d_o + 2e-7 * L)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n,leaf", [(1, 4), (2, 4), (5, 4), (300, 1), (300, 64), (1000, 4)])
def test_lbvh_small_ragged_and_duplicate_inputs(W, dim, n, leaf):
    """Tiny sets, leaf sizes 1 and 64, and sets where every primitive has the
    same Morton code (all centroids in one cell): brute force decides."""
    from paper_2410_18944_amd.api import Lbvh
    rng = np.random.default_rng(7 * n + dim + leaf)
    k = 2 if dim == 2 else 3
    if n == 1000:
        # every primitive the same: one Morton code, a zero-extent bound box
        base = rng.normal(size=(k, dim))
        tris = np.repeat(base[None], n, 0)
    else:
        tris = rng.uniform(-1, 1, (n, k, dim))
    recs = np.zeros((n, 4 if dim == 2 else 12), np.float32)
    recs[:, : k * dim] = tris.reshape(n, -1)
    bv = Lbvh(dim, torch.as_tensor(recs, device="cuda").reshape(-1), leaf_size=leaf)
    torch.cuda.synchronize()
    _check_structure(bv, dim, recs, leaf)
    pts = rng.uniform(-1.5, 1.5, (500, dim)).astype(np.float32)
    d, p = bv.closest(torch.as_tensor(pts, device="cuda"))
    d = d.double().cpu().numpy()
    # brute force in float64 over the float32 primitives
    P = recs[:, : k * dim].reshape(n, k, dim).astype(np.float64)
    X = pts.astype(np.float64)
    if dim == 2:
        a, b = P[:, 0], P[:, 1]
        e = b - a
        t = np.clip(np.einsum("mnd,nd->mn", X[:, None] - a[None], e) / np.maximum(np.sum(e * e, 1), 1e-300), 0, 1)
        c = a[None] + t[..., None] * e[None]
        ref = np.sqrt(np.min(np.sum((X[:, None] - c) ** 2, -1), 1))
    else:
        uniq = P[:1] if n == 1000 else P      # the duplicate set has one distinct triangle
        ref = np.array([min(_pt_tri(x, tri) for tri in uniq) for x in X])
    assert np.all(np.abs(d - ref) <= 1e-5 * ref + 1e-6), np.max(np.abs(d - ref))


def _pt_tri(x, tri):
    """FP64 point-triangle distance by projection onto the plane and the edges."""
    a, b, c = tri
    n = np.cross(b - a, c - a)
    nn = np.dot(n, n)
    best = min(_pt_seg(x, a, b), _pt_seg(x, b, c), _pt_seg(x, c, a))
    if nn > 0:
        p = x - np.dot(x - a, n) / nn * n
        # barycentric inside test
        v0, v1, v2 = b - a, c - a, p - a
        d00, d01, d11, d20, d21 = v0 @ v0, v0 @ v1, v1 @ v1, v2 @ v0, v2 @ v1
        den = d00 * d11 - d01 * d01
        if den > 0:
            v = (d11 * d20 - d01 * d21) / den
            w = (d00 * d21 - d01 * d20) / den
            if v >= 0 and w >= 0 and v + w <= 1:
                best = min(best, abs(np.dot(x - a, n)) / np.sqrt(nn))
    return best


def _pt_seg(x, a, b):
    e = b - a
    t = np.clip(np.dot(x - a, e) / max(np.dot(e, e), 1e-300), 0, 1)
    return np.linalg.norm(x - (a + t * e))


@pytest.mark.parametrize("name,wpp", [("C2", 8), ("C4", 2)])
def test_walks_over_a_gpu_built_dirichlet_hierarchy(W, name, wpp):
    """The solve reading a GPU-built Dirichlet hierarchy (same primitives)
    gives the same walks as over the host-built one: the closest distances
    are identical, and where two primitives tie the closest point is their
    shared point."""
    from paper_2410_18944_amd.api import Lbvh
    s = rounded({"C2": scenes.scene_c2, "C4": scenes.scene_c4}[name]())
    pts = s.points[:: max(1, s.n_points // 4000)]
    geom = W.Geometry.from_scene(s)
    recs = _records(s.dim, s.verts, _dirichlet(s))
    bv = Lbvh(s.dim, torch.as_tensor(recs, device="cuda").reshape(-1), leaf_size=4)
    pb = W.Problem.from_scene(s)
    out = {}
    for which in ("host", "gpu"):
        geom.use_dirichlet_lbvh(bv if which == "gpu" else None)
        n = len(pts)
        wv = torch.empty(n * wpp, dtype=torch.float32, device="cuda")
        ws = torch.empty(n * wpp, dtype=torch.int32, device="cuda")
        W.solve(geom, pb, torch.as_tensor(pts, dtype=torch.float32, device="cuda"), wpp, walk_value=wv,
                walk_steps=ws)
        q = geom.query(torch.as_tensor(pts, dtype=torch.float32, device="cuda"), silhouette=False)
        torch.cuda.synchronize()
        out[which] = (wv.double().cpu().numpy(), ws.cpu().numpy(), q["d_dir"].cpu().numpy())
    geom.use_dirichlet_lbvh(None)
    vh, sh, dh = out["host"]
    vg, sg, dg = out["gpu"]
    np.testing.assert_array_equal(dg, dh)
    same = sg == sh
    say("%s: walks with identical step counts over the GPU-built hierarchy %.5f" % (name, same.mean()))
    assert same.mean() > 0.999
    assert np.all(np.abs(vg - vh)[same] <= 1e-5 * np.maximum(1, np.abs(vh[same])))
