"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the host-only builder validates its input.  No kernel is
launched (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wost.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2410_18944_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2410_18944_amd import build
        build.build()
    return L


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(wost_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["wost_build_bvh", "wost_solve", "wost_guide_infer", "wost_guide_train_step", "wost_query",
                 "wost_tail_pass", "wost_last_error"]:
        assert must in names, must


def test_library_exports_every_declared_symbol(lib):
    L = lib.load()
    missing = [n for n in declared_functions() if getattr(L, n, None) is None]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(lib):
    assert set(declared_functions()) <= set(lib.SIGNATURES), set(declared_functions()) - set(lib.SIGNATURES)


def declared_arity():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"(wost_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_arity_matches_header(lib):
    ar = declared_arity()
    bad = {n: (k, len(lib.SIGNATURES[n][1])) for n, k in ar.items() if len(lib.SIGNATURES[n][1]) != k}
    assert not bad, bad


def _build(lib, dim, verts, prims, bc, leaf=4, brute=0):
    L = lib.load()
    v = np.ascontiguousarray(verts, np.float32)
    p = np.ascontiguousarray(prims, np.int32)
    b = np.ascontiguousarray(bc, np.uint8)
    h = C.c_void_p()
    opts = lib.wost_build_opts(leaf, brute)
    rc = L.wost_build_bvh(dim, v.ctypes.data, v.shape[0], p.ctypes.data, p.shape[0], b.ctypes.data,
                          C.byref(opts), C.byref(h))
    return rc, h


def _info(lib, h):
    info = (C.c_double * 8)()
    assert lib.load().wost_geom_info(h, info) == 0
    return list(info)


@pytest.mark.parametrize("name", ["C1", "C2", "halfdisk", "cube"])
def test_builder_counts_and_depth(lib, name):
    s = scenes.make_scene(name)
    rc, h = _build(lib, s.dim, s.verts, s.prims, s.bc)
    assert rc == 0, lib.load().wost_last_error()
    info = _info(lib, h)
    assert info[0] == s.dim
    assert info[1] == int(np.sum(s.bc == 0))
    assert info[2] == int(np.sum(s.bc == 1))
    # silhouette candidates: Neumann vertices (2D) / Neumann edges (3D)
    N = s.prims[s.bc == 1]
    if s.dim == 2:
        expect = len(np.unique(N.ravel()))
    else:
        e = np.sort(np.concatenate([N[:, [0, 1]], N[:, [1, 2]], N[:, [2, 0]]]), axis=1)
        expect = len(np.unique(e, axis=0)) if len(e) else 0
    assert info[3] == expect
    n_max = max(info[1], info[2], info[3])
    assert info[4] <= int(np.ceil(np.log2(max(n_max, 1) / 4.0))) + 2
    assert info[6] > 0 and int(info[6]) % 256 == 0
    # internal ids map back to caller indices, as a permutation per hierarchy
    ids = [lib.load().wost_geom_prim_index(h, i) for i in range(int(info[1] + info[2]))]
    assert sorted(ids) == list(range(s.prims.shape[0]))
    lib.load().wost_geom_free(h)


def test_builder_brute_force_uses_full_leaves(lib):
    """Brute force packs 64 primitives per leaf (C1: 128 Dirichlet segments ->
    one split), and every hierarchy needs a short traversal stack."""
    s = scenes.scene_c1()
    rc, h = _build(lib, 2, s.verts, s.prims, s.bc, brute=1)
    assert rc == 0
    info = _info(lib, h)
    assert info[4] <= int(np.ceil(np.log2(max(info[1], info[2], 1) / 64.0))) + 1
    assert 1 <= info[7] <= 4
    lib.load().wost_geom_free(h)


@pytest.mark.parametrize("name", ["C2", "cube"])
def test_builder_stack_entries_cover_four_wide_depth(lib, name):
    """A four-wide level spans two binary levels and defers at most three
    children, so the stack needs at most 3 * ceil((depth + 1) / 2) entries."""
    s = scenes.make_scene(name)
    rc, h = _build(lib, s.dim, s.verts, s.prims, s.bc)
    assert rc == 0
    info = _info(lib, h)
    assert 1 <= info[7] <= 3 * int(np.ceil((info[4] + 1) / 2.0)) + 1
    lib.load().wost_geom_free(h)


def test_builder_rejects_bad_input(lib):
    L = lib.load()
    s = scenes.scene_c1()
    rc, _ = _build(lib, 4, s.verts, s.prims, s.bc)
    assert rc == -1 and b"dim" in L.wost_last_error()
    bad = s.prims.copy()
    bad[3, 1] = 999
    rc, _ = _build(lib, 2, s.verts, bad, s.bc)
    assert rc == -1 and b"out of range" in L.wost_last_error()
    deg = s.prims.copy()
    deg[5, 1] = deg[5, 0]
    rc, _ = _build(lib, 2, s.verts, deg, s.bc)
    assert rc == -1 and b"degenerate" in L.wost_last_error()
    bc = s.bc.copy()
    bc[0] = 7
    rc, _ = _build(lib, 2, s.verts, s.prims, bc)
    assert rc == -1
    rc, _ = _build(lib, 2, s.verts, s.prims, s.bc, leaf=0)
    assert rc == -1


def test_upload_and_solve_reject_bad_arguments_without_launch(lib):
    L = lib.load()
    s = scenes.scene_c1()
    rc, h = _build(lib, 2, s.verts, s.prims, s.bc)
    assert rc == 0
    # not uploaded -> ESTATE before any device work
    pb = lib.wost_problem()
    pb.eps = 1e-3
    pb.rr_q = 1.0
    dummy = C.c_void_p(256)
    rc = L.wost_solve(h, C.byref(pb), dummy, 10, 4, 1, 0, None, dummy, dummy, dummy, None, None, None,
                      dummy, 1 << 20, dummy, None)
    assert rc == -4
    assert L.wost_geom_upload(h, None, 0, None) == -1
    assert L.wost_solve_workspace_bytes(h, 100, 8) >= 100 * 8 * 4
    # the wavefront solver takes the same checks, and a workspace that holds
    # every walk's state and its queues
    rc = L.wost_solve_wavefront(h, C.byref(pb), dummy, 10, 4, 1, 0, None, dummy, dummy, dummy, None, None, None,
                                dummy, 1 << 20, dummy, None)
    assert rc == -4
    assert L.wost_solve_wavefront_workspace_bytes(h, 100, 8) >= 100 * 8 * (4 + 20 + 4 * 26)  # 26 state words in 2D
    assert L.wost_set_wavefront_streams(3) < 0 and L.wost_set_wavefront_streams(0) < 0
    assert L.wost_set_wavefront_streams(2) == 0 and L.wost_set_wavefront_streams(1) == 0
    # a GPU-built Dirichlet hierarchy must cover the same primitive count and
    # fit the traversal stack; NULL nodes switch back (host-only checks)
    n_dir = int((s.bc == 0).sum())
    fake = C.c_void_p(4096)
    assert L.wost_geom_use_dirichlet_lbvh(h, fake, 10, fake, fake, n_dir + 1, 5) == -1
    assert L.wost_geom_use_dirichlet_lbvh(h, fake, 10, fake, fake, n_dir, 15) < 0
    assert L.wost_geom_use_dirichlet_lbvh(h, fake, 10, fake, fake, n_dir, 14) == 0
    assert L.wost_geom_use_dirichlet_lbvh(h, None, 0, None, None, 0, 0) == 0
    L.wost_geom_free(h)


def test_lbvh_sizes_validate_and_scale(lib):
    L = lib.load()
    nb, pb, wb = C.c_int64(), C.c_int64(), C.c_int64()
    assert L.wost_lbvh_sizes(4, 10, C.byref(nb), C.byref(pb), C.byref(wb)) < 0
    assert L.wost_lbvh_sizes(3, 0, C.byref(nb), C.byref(pb), C.byref(wb)) < 0
    assert L.wost_lbvh_sizes(3, 1, C.byref(nb), C.byref(pb), C.byref(wb)) == 0
    assert nb.value == 7 * 16 and pb.value == 3 * 16
    assert L.wost_lbvh_sizes(2, 1000, C.byref(nb), C.byref(pb), C.byref(wb)) == 0
    # at most n - 1 four-wide nodes of 5 float4; one float4 per segment
    assert nb.value == 999 * 5 * 16 and pb.value == 1000 * 16 and wb.value >= 1000 * 4 * 4
    assert L.wost_lbvh_build(2, None, 1000, 4, None, None, None, None, None, None, 0, None) < 0


def test_guide_create_validates_config(lib):
    L = lib.load()
    from paper_2410_18944_amd.guide import GuideConfig
    h = C.c_void_p()
    good = GuideConfig(dim=2, levels=8, log2_table=16, n_min=16, n_max=1024, n_hidden=2, K=8,
                       aabb_lo=(-1, -1), aabb_hi=(1, 1))
    c = good.to_c()
    assert L.wost_guide_create(C.byref(c), C.byref(h)) == 0
    P = L.wost_guide_param_count(h)
    assert P == 8 * (1 << 16) * 2 + 16 * 64 + 64 * 64 + 64 * 33
    assert L.wost_guide_shadow_bytes(h) >= 2 * P
    L.wost_guide_free(h)
    for bad in [dict(levels=7), dict(hidden=32), dict(K=0), dict(dim=4), dict(feats=4)]:
        cfg = GuideConfig(**{**good.__dict__, **bad})
        c = cfg.to_c()
        assert L.wost_guide_create(C.byref(c), C.byref(h)) < 0


def test_device_build_workspace_validates_and_scales(lib):
    """The device build's size query and argument checks run on the host
    (no kernel is launched before they pass)."""
    L = lib.load()
    ws = C.c_int64()
    opts = lib.wost_build_opts(4, 0)
    assert L.wost_build_bvh_device_workspace(4, 10, 10, None, C.byref(ws)) == -1
    assert L.wost_build_bvh_device_workspace(2, 10, 0, None, C.byref(ws)) == -1
    assert L.wost_build_bvh_device_workspace(2, 10, 10, C.byref(lib.wost_build_opts(0, 0)), C.byref(ws)) == -1
    assert L.wost_build_bvh_device_workspace(2, 10, 1 << 26, None, C.byref(ws)) < 0
    sizes = []
    for n in (1, 100, 10000):
        assert L.wost_build_bvh_device_workspace(3, 3 * n, n, C.byref(opts), C.byref(ws)) == 0
        sizes.append(ws.value)
    assert sizes[0] > 0 and sizes[0] < sizes[1] < sizes[2]
    assert sizes[2] < 2000 * 10000   # linear, about 1 KB per triangle
    h = C.c_void_p()
    fake = C.c_void_p(4096)
    assert L.wost_build_bvh_device(2, None, 10, fake, 10, fake, None, fake, 1 << 30, None, C.byref(h)) == -1
    assert L.wost_build_bvh_device(2, fake, 10, fake, 10, fake, C.byref(lib.wost_build_opts(4, 1)), fake, 1 << 30,
                                   None, C.byref(h)) < 0
    assert L.wost_build_bvh_device(2, fake, 10, fake, 10, fake, None, fake, 16, None, C.byref(h)) == -2
    assert L.wost_build_bvh_device(2, fake, 10, fake, 10, fake, None, C.c_void_p(4096 + 8), 1 << 30, None,
                                   C.byref(h)) == -1
    assert not h.value
