"""The geometry image built on the GPU (wost_build_bvh_device) against the
host builder (wost_build_bvh): the two images are compared byte for byte
(Dirichlet, Neumann and silhouette hierarchies with measures, normal cones
and convex pieces, primitive records, id tables), handle statistics and id
maps agree, and walks over the two images give bit-identical estimates.
Invalid inputs are rejected by the device build's own checks."""
import time

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_18944_amd as W
    return W


def _both(W, dim, verts, prims, bc, leaf=4):
    t0 = time.perf_counter()
    gh = W.Geometry(dim, verts, prims, bc, leaf_size=leaf, build="host")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gg = W.Geometry(dim, verts, prims, bc, leaf_size=leaf, build="gpu")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say("  host build %.3f s, gpu build %.3f s, %d bytes" % (t1 - t0, t2 - t1, gh.nbytes))
    return gh, gg


def _compare(W, gh, gg, n_prims):
    assert gh.info == gg.info, (gh.info, gg.info)
    a = gh.image().cpu().numpy()
    b = gg.image().cpu().numpy()
    assert a.shape == b.shape
    diff = np.flatnonzero(a != b)
    if diff.size:
        for o in np.unique(diff // 16)[:6]:
            say("  differ at 16-byte word %d: host %s gpu %s / host %s gpu %s" % (
                o, a[16 * o:16 * o + 16].view(np.float32), b[16 * o:16 * o + 16].view(np.float32),
                a[16 * o:16 * o + 16].view(np.int32), b[16 * o:16 * o + 16].view(np.int32)))
    assert diff.size == 0, "first differing byte %d of %d (%d differ)" % (diff[0], a.size, diff.size)
    lib = W._lib.load()
    n_int = gh.info["n_dirichlet"] + gh.info["n_neumann"]
    ids = np.unique(np.r_[0, n_int - 1, np.linspace(0, max(n_int - 1, 0), 97).astype(int)])
    for i in ids:
        assert lib.wost_geom_prim_index(gh.h, int(i)) == lib.wost_geom_prim_index(gg.h, int(i))


@pytest.mark.parametrize("name", ["C1", "C2", "halfdisk", "cube", "cube-neumann-face", "halfsphere", "sphere-sources",
                                  "C4"])
def test_device_image_equals_host_image(W, name):
    s = scenes.make_scene(name)
    say("geometry build", name, s.dim, "D", len(s.prims), "primitives,", int(s.bc.sum()), "Neumann")
    gh, gg = _both(W, s.dim, s.verts, s.prims, s.bc)
    _compare(W, gh, gg, len(s.prims))


@pytest.mark.parametrize("leaf", [1, 3, 64])
def test_device_image_equals_host_image_leaf_sizes(W, leaf):
    s = scenes.make_scene("C2")
    say("geometry build C2 leaf", leaf)
    gh, gg = _both(W, s.dim, s.verts, s.prims, s.bc, leaf=leaf)
    _compare(W, gh, gg, len(s.prims))


def _polygon(n, r=1.0, jitter=0.0, seed=0):
    rng = np.random.default_rng(seed)
    t = np.linspace(0, 2 * np.pi, n, endpoint=False)
    rr = r * (1 + jitter * rng.uniform(-1, 1, n))
    v = np.stack([rr * np.cos(t), rr * np.sin(t)], 1)
    p = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1).astype(np.int32)
    return v, p


@pytest.mark.parametrize("case", ["one-neumann", "two-dirichlet", "all-neumann-5", "all-dirichlet", "ragged-mixed",
                                  "duplicate-centroids", "reversed-segment", "open-chain"])
def test_device_image_small_and_degenerate_layouts(W, case):
    """Tiny and ragged sets: single primitives, one empty class, equal
    centroids (ties broken by index), inconsistently oriented and open
    chains (no links, boundary candidates)."""
    rng = np.random.default_rng(5)
    if case == "one-neumann":
        v, p = _polygon(3)
        p, bc = p[:1], np.array([1], np.uint8)
    elif case == "two-dirichlet":
        v, p = _polygon(3)
        p, bc = p[:2], np.zeros(2, np.uint8)
    elif case == "all-neumann-5":
        v, p = _polygon(5)
        bc = np.ones(5, np.uint8)
    elif case == "all-dirichlet":
        v, p = _polygon(301, jitter=0.2, seed=3)
        bc = np.zeros(301, np.uint8)
    elif case == "ragged-mixed":
        v, p = _polygon(1001, jitter=0.3, seed=4)
        bc = (rng.uniform(size=1001) < 0.6).astype(np.uint8)
    elif case == "duplicate-centroids":
        # 200 copies of the same four segments: every centroid repeats
        v, p0 = _polygon(4)
        p = np.tile(p0, (200, 1))
        bc = (np.arange(800) % 3 == 0).astype(np.uint8)
    elif case == "reversed-segment":
        v, p = _polygon(64, jitter=0.1, seed=6)
        p[7] = p[7][::-1]
        bc = np.ones(64, np.uint8)
    else:
        v, p = _polygon(64, jitter=0.1, seed=7)
        p, bc = p[:40], np.ones(40, np.uint8)
    say("geometry build", case, len(p))
    gh, gg = _both(W, 2, v, p, bc)
    _compare(W, gh, gg, len(p))


def test_device_image_equals_host_image_3d_open_and_duplicated(W):
    """A 3D mesh with boundary edges (an open hemisphere, Neumann) and a
    duplicated Dirichlet copy of part of it."""
    s = scenes.make_scene("sphere-sources")
    keep = s.verts[s.prims].mean(1)[:, 2] > -0.2
    prims = s.prims[keep]
    bc = np.ones(len(prims), np.uint8)
    extra = prims[: len(prims) // 3]
    prims = np.concatenate([prims, extra])
    bc = np.concatenate([bc, np.zeros(len(extra), np.uint8)])
    say("geometry build open hemisphere", len(prims))
    gh, gg = _both(W, 3, s.verts, prims, bc)
    _compare(W, gh, gg, len(prims))


def test_device_build_at_full_size(W):
    """The 1M-triangle mesh: identical image, and the device build's time."""
    s = scenes.scene_c5(n_random=16)
    say("geometry build C5", len(s.prims))
    gh, gg = _both(W, s.dim, s.verts, s.prims, s.bc)
    _compare(W, gh, gg, len(s.prims))


@pytest.mark.parametrize("name", ["C2", "C4"])
def test_walks_over_device_image_identical(W, name):
    s = scenes.make_scene(name)
    rng = np.random.default_rng(12)
    pts = s.points[rng.choice(s.n_points, min(s.n_points, 4096), replace=False)]
    tp = torch.as_tensor(np.asarray(pts, np.float32), device="cuda")
    out = []
    for build in ("host", "gpu"):
        geom = W.Geometry(s.dim, s.verts, s.prims, s.bc, build=build)
        pb = W.Problem.from_scene(s)
        wv = torch.empty(len(pts) * 8, dtype=torch.float32, device="cuda")
        ws = torch.empty(len(pts) * 8, dtype=torch.int32, device="cuda")
        acc = W.solve(geom, pb, tp, 8, seed=77, walk_value=wv, walk_steps=ws)
        torch.cuda.synchronize()
        m, se, _ = acc.estimates()
        out.append((m.cpu().numpy(), wv.cpu().numpy(), ws.cpu().numpy()))
    say("walks", name, "steps", int(out[0][2].sum()))
    np.testing.assert_array_equal(out[0][2], out[1][2])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][0], out[1][0])


@pytest.mark.parametrize("bad", ["bc", "vertex", "degenerate", "nonfinite"])
def test_device_build_rejects_invalid_input(W, bad):
    v, p = _polygon(16)
    bc = np.ones(16, np.uint8)
    if bad == "bc":
        bc[5] = 2
    elif bad == "vertex":
        p = p.copy()
        p[9, 1] = 99
    elif bad == "degenerate":
        p = p.copy()
        p[3, 1] = p[3, 0]
    else:
        v = v.copy()
        v[2, 0] = np.nan
    with pytest.raises(RuntimeError) as e:
        W.Geometry(2, v, p, bc, build="gpu")
    say("rejected:", e.value)
    with pytest.raises(RuntimeError):
        W.Geometry(2, v, p, bc, build="host")
