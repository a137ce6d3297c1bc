"""Python surface over the C ABI: geometry, problem, solve, guide.

Device memory comes from torch tensors on the current HIP device and every
launch goes to torch's current stream; the library allocates nothing.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

N_COUNTERS = 8
COUNTER_NAMES = ["steps", "walks", "truncated", "rr_killed", "nonfinite", "records", "records_dropped", "unused"]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _field(desc, keep):
    """(kind, params) with kind an int code or a name -> wost_field."""
    kind, params = desc
    if isinstance(kind, str):
        kind = L.FIELD[kind]
    arr = np.ascontiguousarray(np.asarray(params, np.float32).ravel())
    keep.append(arr)
    n = 0
    if kind == L.FIELD["const"]:
        n = 1
    elif kind == L.FIELD["gauss_sum"]:
        rows = np.asarray(params)
        n = int(rows.shape[0]) if rows.ndim == 2 else 0
    ptr = arr.ctypes.data_as(C.POINTER(C.c_float)) if arr.size else None
    return L.wost_field(int(kind), n, ptr)


class Geometry:
    """Boundary hierarchies in a torch buffer, built on the host
    (``build="host"``, wost_build_bvh) or on the GPU from device copies of the
    inputs (``build="gpu"``, wost_build_bvh_device); both give the same image."""

    def __init__(self, dim, verts, prims, bc, leaf_size=4, brute_force=False, device=None, build="host"):
        lib = L.load()
        self.dim = int(dim)
        opts = L.wost_build_opts(int(leaf_size), 1 if brute_force else 0)
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        h = C.c_void_p()
        ws = None
        if build == "host":
            v = np.ascontiguousarray(verts, np.float32)
            p = np.ascontiguousarray(prims, np.int32)
            b = np.ascontiguousarray(bc, np.uint8)
            L.check(lib.wost_build_bvh(self.dim, v.ctypes.data, v.shape[0], p.ctypes.data, p.shape[0],
                                       b.ctypes.data, C.byref(opts), C.byref(h)), "wost_build_bvh")
        elif build == "gpu":
            v = torch.as_tensor(np.ascontiguousarray(verts, np.float32), device=dev).contiguous()
            p = torch.as_tensor(np.ascontiguousarray(prims, np.int32), device=dev).contiguous()
            b = torch.as_tensor(np.ascontiguousarray(bc, np.uint8), device=dev).contiguous()
            need = C.c_int64()
            L.check(lib.wost_build_bvh_device_workspace(self.dim, v.shape[0], p.shape[0], C.byref(opts),
                                                        C.byref(need)), "wost_build_bvh_device_workspace")
            ws = torch.empty(need.value + 256, dtype=torch.uint8, device=dev)
            ws_base = ws.data_ptr() + (-ws.data_ptr()) % 256
            L.check(lib.wost_build_bvh_device(self.dim, v.data_ptr(), v.shape[0], p.data_ptr(), p.shape[0],
                                              b.data_ptr(), C.byref(opts), C.c_void_p(ws_base), need.value,
                                              _stream(), C.byref(h)), "wost_build_bvh_device")
        else:
            raise ValueError("build must be 'host' or 'gpu'")
        self.h = h
        nbytes = lib.wost_geom_device_bytes(h)
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.buf.data_ptr()) % 256
        self._base = self.buf.data_ptr() + off
        self._off = off
        self.nbytes = int(nbytes)
        L.check(lib.wost_geom_upload(h, C.c_void_p(self._base), nbytes, _stream()), "wost_geom_upload")
        del ws
        info = (C.c_double * 8)()
        L.check(lib.wost_geom_info(h, info), "wost_geom_info")
        self.info = dict(dim=int(info[0]), n_dirichlet=int(info[1]), n_neumann=int(info[2]),
                         n_silhouette=int(info[3]), max_depth=int(info[4]), diag=float(info[5]),
                         bytes=int(info[6]))

    def image(self):
        """The uploaded device image as a uint8 tensor view."""
        return self.buf[self._off:self._off + self.nbytes]

    @classmethod
    def from_scene(cls, scene, **kw):
        return cls(scene.dim, scene.verts, scene.prims, scene.bc, **kw)

    def __del__(self):
        # at interpreter shutdown the binding module may already be torn down
        lib = getattr(L, "_lib", None) if L is not None else None
        if getattr(self, "h", None) is not None and lib is not None:
            lib.wost_geom_free(self.h)
            self.h = None

    def use_dirichlet_lbvh(self, bv=None):
        """Walk and query over a GPU-built hierarchy ``bv`` (an ``Lbvh`` over
        the same Dirichlet primitives) instead of the host-built one; None
        switches back."""
        lib = L.load()
        if bv is None:
            L.check(lib.wost_geom_use_dirichlet_lbvh(self.h, None, 0, None, None, 0, 0), "wost_geom_use_dirichlet_lbvh")
        else:
            L.check(lib.wost_geom_use_dirichlet_lbvh(self.h, _ptr(bv.nodes), bv.n_nodes, _ptr(bv.prims),
                                                     _ptr(bv.orig), bv.n, bv.levels), "wost_geom_use_dirichlet_lbvh")
        self._dir_lbvh = bv      # keeps the buffers alive while in use

    def neumann_sample(self, pts, radius, uniforms, on_prim=None):
        """The walk's Neumann-sample step at given states (wost_neumann_sample):
        returns dict(prim, prob, z, accepted) as tensors."""
        lib = L.load()
        pts = pts.contiguous()
        n = pts.shape[0]
        dev = pts.device
        out = dict(prim=torch.empty(n, dtype=torch.int32, device=dev), prob=torch.empty(n, dtype=torch.float32, device=dev),
                   z=torch.empty(n, self.dim, dtype=torch.float32, device=dev),
                   accepted=torch.empty(n, dtype=torch.int32, device=dev))
        op = on_prim.contiguous() if on_prim is not None else None
        L.check(lib.wost_neumann_sample(self.h, _ptr(pts), n, _ptr(op), _ptr(radius.contiguous()),
                                        _ptr(uniforms.contiguous()), _ptr(out["prim"]), _ptr(out["prob"]),
                                        _ptr(out["z"]), _ptr(out["accepted"]), _stream()), "wost_neumann_sample")
        return out

    def query(self, pts, dirichlet=True, silhouette=True, ray_dir=None, ray_tmax=None, on_prim=None):
        lib = L.load()
        pts = pts.contiguous()
        n = pts.shape[0]
        dev = pts.device
        out = {}
        d_dir = torch.empty(n, dtype=torch.float32, device=dev) if dirichlet else None
        xbar = torch.empty(n, self.dim, dtype=torch.float32, device=dev) if dirichlet else None
        d_sil = torch.empty(n, dtype=torch.float32, device=dev) if silhouette else None
        ray_t = ray_prim = None
        if ray_dir is not None:
            ray_dir = ray_dir.contiguous()
            ray_tmax = torch.as_tensor(ray_tmax, dtype=torch.float32, device=dev).expand(n).contiguous()
            ray_t = torch.empty(n, dtype=torch.float32, device=dev)
            ray_prim = torch.empty(n, dtype=torch.int32, device=dev)
        if on_prim is not None:
            on_prim = torch.as_tensor(on_prim, dtype=torch.int32, device=dev).contiguous()
        L.check(lib.wost_query(self.h, _ptr(pts), n, _ptr(on_prim), _ptr(d_dir), _ptr(xbar), _ptr(d_sil), _ptr(ray_dir),
                               _ptr(ray_tmax), _ptr(ray_t), _ptr(ray_prim), _stream()), "wost_query")
        if dirichlet:
            out.update(d_dir=d_dir, xbar=xbar)
        if silhouette:
            out["d_sil"] = d_sil
        if ray_dir is not None:
            out.update(ray_t=ray_t, ray_prim=ray_prim)
        return out


class Problem:
    """Mirror of wost_problem; fields are (kind, params) pairs."""

    def __init__(self, g, h=("zero", ()), f=("zero", ()), eps=1e-3, r_min=0.0, max_steps=4096, rr_start=128,
                 rr_q=0.99, sampling="uniform", c_fixed=0.5, reflect=True):
        self.g, self.h, self.f = g, h, f
        self.eps, self.r_min, self.max_steps, self.rr_start, self.rr_q = eps, r_min, max_steps, rr_start, rr_q
        self.sampling, self.c_fixed, self.reflect = sampling, c_fixed, reflect

    def image(self):
        """The uploaded device image as a uint8 tensor view."""
        return self.buf[self._off:self._off + self.nbytes]

    @classmethod
    def from_scene(cls, scene, **kw):
        args = dict(g=scene.g, h=scene.h, f=scene.f, eps=scene.eps, max_steps=scene.max_steps,
                    rr_start=min(scene.rr_start, 2 ** 31 - 1), rr_q=scene.rr_q)
        args.update(kw)
        return cls(**args)

    def to_c(self):
        keep = []
        s = self.sampling
        s = L.SAMPLING[s] if isinstance(s, str) else int(s)
        pb = L.wost_problem(_field(self.g, keep), _field(self.h, keep), _field(self.f, keep),
                            float(self.eps), float(self.r_min), int(self.max_steps), int(self.rr_start),
                            float(self.rr_q), s, float(self.c_fixed), 1 if self.reflect else 0)
        return pb, keep


class Records:
    """Training-record buffer (structure of arrays, see wost_records)."""

    def __init__(self, dim, capacity, device=None):
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.dim = dim
        self.capacity = int(capacity)
        self.nf = 3 * dim + 5
        self.data = torch.zeros(self.nf, self.capacity, dtype=torch.float32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)

    def reset(self):
        self.count.zero_()

    def to_c(self):
        return L.wost_records(C.c_void_p(self.data.data_ptr()), self.capacity, C.c_void_p(self.count.data_ptr()))

    def n(self):
        return min(int(self.count.item()), self.capacity)

    def fields(self, n=None):
        n = self.n() if n is None else n
        d = self.dim
        D = self.data[:, :n]
        return dict(x=D[0:d].T, nu=D[d:2 * d].T, n=D[2 * d:3 * d].T, p_sample=D[3 * d], prefix=D[3 * d + 1],
                    t_next=D[3 * d + 2], slot=D[3 * d + 3].view(torch.int32), p_t=D[3 * d + 4])


class Accumulator:
    """Per-point FP64 sums (accumulated across calls) and run counters."""

    def __init__(self, n_points, device=None):
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.sum = torch.zeros(n_points, dtype=torch.float64, device=dev)
        self.sum_sq = torch.zeros(n_points, dtype=torch.float64, device=dev)
        self.count = torch.zeros(n_points, dtype=torch.int64, device=dev)
        self.counters = torch.zeros(N_COUNTERS, dtype=torch.int64, device=dev)

    def estimates(self):
        n = self.count.double()
        mean = self.sum / n
        var = torch.clamp(self.sum_sq / n - mean * mean, min=0.0) * n / torch.clamp(n - 1, min=1)
        return mean, torch.sqrt(var / n), n

    def stats(self):
        c = self.counters.cpu().numpy()
        return {k: int(v) for k, v in zip(COUNTER_NAMES, c)}


ENGINES = {"persistent": ("wost_solve", "wost_solve_workspace_bytes"),
           "wavefront": ("wost_solve_wavefront", "wost_solve_wavefront_workspace_bytes")}


def solve(geom, problem, pts, wpp, seed=18944, walk_offset=0, guide=None, acc=None, walk_value=None,
          walk_steps=None, records=None, workspace=None, engine="persistent"):
    """Launch a solve on the current stream; returns the Accumulator.
    ``engine``: "persistent" (wost_solve, the fused persistent kernel) or
    "wavefront" (wost_solve_wavefront, one kernel per stage; it waits for
    the stream while it runs)."""
    lib = L.load()
    if engine not in ENGINES:
        raise ValueError("engine must be one of %s" % sorted(ENGINES))
    fn, ws_fn = ENGINES[engine]
    pts = pts.contiguous()
    n = pts.shape[0]
    if acc is None:
        acc = Accumulator(n, pts.device)
    need = max(int(getattr(lib, ws_fn)(geom.h, n, int(wpp))), 256)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=pts.device)
    pb, keep = problem.to_c()
    rec = records.to_c() if records is not None else None
    L.check(getattr(lib, fn)(geom.h, C.byref(pb), _ptr(pts), n, int(wpp), int(seed), int(walk_offset),
                             guide.h if guide is not None else None, _ptr(acc.sum), _ptr(acc.sum_sq),
                             _ptr(acc.count), _ptr(walk_value), _ptr(walk_steps),
                             C.byref(rec) if rec is not None else None, _ptr(workspace), workspace.numel(),
                             _ptr(acc.counters), _stream()), fn)
    del keep
    return acc


class Lbvh:
    """A closest-point hierarchy built on the GPU (wost_lbvh_build) over
    primitives given as a device float32 tensor of float4 records (2D: one
    (ax, ay, bx, by) per segment; 3D: three per triangle)."""

    def __init__(self, dim, prims, leaf_size=4):
        lib = L.load()
        prims = prims.contiguous()
        per = 4 if dim == 2 else 12
        n = prims.numel() // per
        nb, pb, wb = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(lib.wost_lbvh_sizes(int(dim), n, C.byref(nb), C.byref(pb), C.byref(wb)), "wost_lbvh_sizes")
        dev = prims.device
        self.dim, self.n = dim, n
        self.nodes = torch.empty(nb.value // 4, dtype=torch.float32, device=dev)
        self.prims = torch.empty(pb.value // 4, dtype=torch.float32, device=dev)
        self.orig = torch.empty(n, dtype=torch.int32, device=dev)
        ws = torch.empty(wb.value + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        nn, lv = C.c_int32(), C.c_int32()
        L.check(lib.wost_lbvh_build(int(dim), _ptr(prims), n, int(leaf_size), _ptr(self.nodes), _ptr(self.prims),
                                    _ptr(self.orig), C.byref(nn), C.byref(lv), C.c_void_p(ws.data_ptr() + off),
                                    wb.value, _stream()), "wost_lbvh_build")
        self.n_nodes, self.levels = nn.value, lv.value

    def closest(self, pts):
        pts = pts.contiguous()
        m = pts.shape[0]
        dist = torch.empty(m, dtype=torch.float32, device=pts.device)
        prim = torch.empty(m, dtype=torch.int32, device=pts.device)
        L.check(L.load().wost_lbvh_closest(self.dim, _ptr(self.nodes), self.n_nodes, _ptr(self.prims),
                                           _ptr(self.orig), self.n, self.levels, _ptr(pts), m, _ptr(dist),
                                           _ptr(prim), _stream()), "wost_lbvh_closest")
        return dist, prim


def set_wavefront_streams(n_streams):
    """Streams of guided wavefront solves: 1 (default) or 2 (the network on
    its own stream, overlapping the other half's geometric stages)."""
    L.check(L.load().wost_set_wavefront_streams(int(n_streams)), "wost_set_wavefront_streams")


def set_walk_pool(slots_per_wave=0, refill_batch=0):
    """Walk slots per persistent wave (multiple of 64; 0 = default 384) and
    the number of finished lanes that refill together (0 = default 32)."""
    L.check(L.load().wost_set_walk_pool(int(slots_per_wave), int(refill_batch)), "wost_set_walk_pool")


def set_launch(waves_per_cu):
    L.check(L.load().wost_set_launch(int(waves_per_cu)), "wost_set_launch")


COST_QUERIES = ["closest_dirichlet", "silhouette", "neumann_sample", "neumann_visibility", "source_visibility",
                "first_hit"]


def set_cost_counters(counters):
    """Enable (int64 device tensor of 18) or disable (None) traversal-cost counting."""
    if counters is not None and counters.numel() < 18:
        raise ValueError("cost counters need 18 int64 entries")
    L.check(L.load().wost_set_cost_counters(_ptr(counters) if counters is not None else None),
            "wost_set_cost_counters")


def cost_report(counters, steps):
    """Per query: nodes and primitives per walk step (lane sums), and the
    wave-level iteration count relative to a perfectly packed wave
    (64 x wave iterations / lane node visits; 1 means no divergence loss)."""
    c = counters.cpu().numpy().astype(float)
    return {q: dict(nodes_per_step=c[2 * i] / steps, prims_per_step=c[2 * i + 1] / steps,
                    wave_iters=c[12 + i], divergence=64.0 * c[12 + i] / max(c[2 * i], 1.0))
            for i, q in enumerate(COST_QUERIES)}
