"""FP64 CPU oracle for walk on stars -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here; the two share
no code.  The only common inputs are the seeded scene arrays from ``scenes``.

``wost_oracle.c`` is a brute-force, uniform-sampling FP64 WoSt (built with gcc
+ OpenMP by :func:`build`); ``guide_ref`` holds FP64 reference definitions of
the guiding distribution (vMF mixture, reflection, MIS, samplers, network and
training loss).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wost_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-misleading-indentation", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("params", C.POINTER(C.c_double))]


class _Problem(C.Structure):
    _fields_ = [("g", _Field), ("h", _Field), ("f", _Field),
                ("eps", C.c_double), ("r_min", C.c_double),
                ("max_steps", C.c_int32), ("rr_start", C.c_int32), ("rr_q", C.c_double)]


def _bind(lib):
    """Declare the argument and result types of the oracle's C entry points."""
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    lib.or_scene_create.restype = P
    lib.or_scene_create.argtypes = [C.c_int, dp, C.c_int64, C.POINTER(C.c_int32), C.c_int64,
                                    C.POINTER(C.c_uint8)]
    lib.or_scene_free.argtypes = [P]
    lib.or_scene_set_tolerance.argtypes = [P, C.c_double]
    lib.or_scene_n_silhouette_candidates.restype = C.c_int64
    lib.or_scene_n_silhouette_candidates.argtypes = [P]
    lib.or_solve.restype = C.c_int
    lib.or_solve.argtypes = [P, C.POINTER(_Problem), dp, C.c_int64, C.POINTER(C.c_int64), C.c_int32, C.c_uint64, C.c_uint64,
                             dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                             dp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int]
    lib.or_walk_trace.restype = C.c_int32
    lib.or_walk_trace.argtypes = [P, C.POINTER(_Problem), dp, C.c_uint64, C.c_uint32, C.c_uint32,
                                  dp, dp, C.c_int32, dp, dp, C.POINTER(C.c_int32)]
    lib.or_first_step.restype = C.c_int
    lib.or_first_step.argtypes = [P, C.POINTER(_Problem), dp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, dp]
    lib.or_closest_dirichlet.argtypes = [P, dp, C.c_int64, dp, dp]
    lib.or_silhouette.argtypes = [P, dp, C.c_int64, C.POINTER(C.c_int64), dp]
    lib.or_ray_neumann.argtypes = [P, dp, dp, dp, C.c_int64, dp, C.POINTER(C.c_int64)]
    lib.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    lib.or_philox4x32_10_batch.argtypes = [C.POINTER(C.c_uint32), C.c_int64, C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
    lib.or_green_ball.restype = C.c_double
    lib.or_green_ball.argtypes = [C.c_int, C.c_double, C.c_double]
    lib.or_field_value.restype = C.c_double
    lib.or_field_value.argtypes = [C.c_int, C.c_int, dp, C.c_int, dp]
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _bind(C.CDLL(_LIB))
    return _lib


def source_text() -> str:
    """The oracle's C source (for tests that compile altered copies)."""
    with open(_SRC) as fh:
        return fh.read()


def load_variant(src: str, directory: str, tag: str):
    """Compile C source text ``src`` (an altered copy of the oracle, used by
    the tests that check a pin fails under a planted mistake) into
    ``directory`` and return its bound library handle, for
    ``OracleScene(..., lib=...)``."""
    c_path = os.path.join(directory, "oracle_%s.c" % tag)
    so_path = os.path.join(directory, "liboracle_%s.so" % tag)
    with open(c_path, "w") as fh:
        fh.write(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", c_path, "-o", so_path, "-lm"],
                   check=True)
    return _bind(C.CDLL(so_path))


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib.or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def philox_batch(ctr, key):
    """ctr uint32 [n, 4] -> Philox4x32-10 outputs [n, 4]."""
    lib = _load()
    c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros_like(c)
    lib.or_philox4x32_10_batch(_ptr(c, C.c_uint32), c.shape[0], _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def green_ball(d, r, rho):
    return _load().or_green_ball(d, r, rho)


def field_value(field, dim, x):
    kind, params = field
    params = np.ascontiguousarray(params, np.float64).ravel()
    n = int(params.size // (2 + dim)) if kind == 6 else int(params.size)
    x = np.ascontiguousarray(x, np.float64)
    return _load().or_field_value(int(kind), n, _ptr(params, C.c_double) if params.size else None,
                                  dim, _ptr(x, C.c_double))


class OracleScene:
    """Exhaustive FP64 scene built from the seeded arrays of a ``scenes.Scene``."""

    def __init__(self, scene, tau_rel=None, lib=None):
        lib = lib if lib is not None else _load()
        self._L = lib
        self.scene = scene
        self.dim = scene.dim
        self._v = np.ascontiguousarray(scene.verts, np.float64)
        self._p = np.ascontiguousarray(scene.prims, np.int32)
        self._b = np.ascontiguousarray(scene.bc, np.uint8)
        self.h = lib.or_scene_create(self.dim, _ptr(self._v, C.c_double), self._v.shape[0],
                                     _ptr(self._p, C.c_int32), self._p.shape[0], _ptr(self._b, C.c_uint8))
        if not self.h:
            raise ValueError("or_scene_create failed")
        if tau_rel is not None:
            lib.or_scene_set_tolerance(self.h, float(tau_rel))
        self._keep = []

    def __del__(self):
        if getattr(self, "h", None) and getattr(self, "_L", None) is not None:
            self._L.or_scene_free(self.h)
            self.h = None

    @property
    def n_silhouette_candidates(self):
        return self._L.or_scene_n_silhouette_candidates(self.h)

    def _problem(self, eps=None, r_min=None, max_steps=None, rr_start=None, rr_q=None):
        s = self.scene
        keep = []

        def fld(fd):
            kind, params = fd
            params = np.ascontiguousarray(params, np.float64).ravel()
            keep.append(params)
            n = int(params.size // (2 + self.dim)) if kind == 6 else int(params.size)
            return _Field(int(kind), n, _ptr(params, C.c_double) if params.size else None)

        eps = s.eps if eps is None else eps
        pb = _Problem(fld(s.g), fld(s.h), fld(s.f), eps, eps if r_min is None else r_min,
                      s.max_steps if max_steps is None else max_steps,
                      s.rr_start if rr_start is None else rr_start,
                      s.rr_q if rr_q is None else rr_q)
        self._keep = keep
        return pb

    def solve(self, points=None, wpp=None, seed=18944, walk_offset=0, per_walk=False,
              nthreads=0, point_ids=None, **problem_kw):
        lib = self._L
        pts = np.ascontiguousarray(self.scene.points if points is None else points, np.float64)
        n = pts.shape[0]
        wpp = self.scene.wpp if wpp is None else wpp
        pb = self._problem(**problem_kw)
        su = np.zeros(n)
        sq = np.zeros(n)
        cnt = np.zeros(n, np.int64)
        st = np.zeros(n, np.int64)
        wv = ws = wst = None
        if per_walk:
            wv = np.zeros(n * wpp)
            ws = np.zeros(n * wpp, np.int32)
            wst = np.zeros(n * wpp, np.int32)
        ids = None if point_ids is None else np.ascontiguousarray(point_ids, np.int64)
        if ids is not None and ids.shape != (n,):
            raise ValueError("point_ids must hold one id per point")
        rc = lib.or_solve(self.h, C.byref(pb), _ptr(pts, C.c_double), n,
                          _ptr(ids, C.c_int64) if ids is not None else None, wpp, seed, walk_offset,
                          _ptr(su, C.c_double), _ptr(sq, C.c_double), _ptr(cnt, C.c_int64),
                          _ptr(st, C.c_int64),
                          _ptr(wv, C.c_double) if per_walk else None,
                          _ptr(ws, C.c_int32) if per_walk else None,
                          _ptr(wst, C.c_int32) if per_walk else None, nthreads)
        if rc != 0:
            raise RuntimeError("or_solve failed")
        out = {"sum": su, "sumsq": sq, "count": cnt, "steps": st}
        if per_walk:
            out.update(walk_value=wv, walk_steps=ws, walk_status=wst)
        return out

    def walk_trace(self, x0, p, j, seed=18944, cap=1 << 16, **problem_kw):
        lib = self._L
        pb = self._problem(**problem_kw)
        x0 = np.ascontiguousarray(x0, np.float64)
        c = np.zeros(cap)
        w = np.zeros(cap)
        val = C.c_double()
        term = C.c_double()
        status = C.c_int32()
        n = lib.or_walk_trace(self.h, C.byref(pb), _ptr(x0, C.c_double), seed, p, j,
                              _ptr(c, C.c_double), _ptr(w, C.c_double), cap,
                              C.byref(val), C.byref(term), C.byref(status))
        return {"c": c[:n], "w": w[:n], "value": val.value, "terminal": term.value,
                "status": status.value}

    def first_step(self, x0, n, p=0, j0=0, seed=18944, **problem_kw):
        """Per walk, the first star's contribution N_0 + S_0 (0 if the walk
        ends at once) for walks j0 .. j0 + n - 1 of point p started at x0."""
        pb = self._problem(**problem_kw)
        x0 = np.ascontiguousarray(x0, np.float64)
        out = np.zeros(int(n))
        rc = self._L.or_first_step(self.h, C.byref(pb), _ptr(x0, C.c_double), seed, p, j0, int(n),
                                   _ptr(out, C.c_double))
        if rc != 0:
            raise RuntimeError("or_first_step failed")
        return out

    def closest_dirichlet(self, x):
        x = np.ascontiguousarray(x, np.float64)
        n = x.shape[0]
        d = np.zeros(n)
        xb = np.zeros_like(x)
        self._L.or_closest_dirichlet(self.h, _ptr(x, C.c_double), n, _ptr(d, C.c_double),
                                     _ptr(xb, C.c_double))
        return d, xb

    def silhouette(self, x, on_prim=None):
        """on_prim: optional per-point primitive index the point lies on (-1 =
        none); that primitive then faces its point from the front."""
        x = np.ascontiguousarray(x, np.float64)
        d = np.zeros(x.shape[0])
        op = None if on_prim is None else np.ascontiguousarray(on_prim, np.int64)
        self._L.or_silhouette(self.h, _ptr(x, C.c_double), x.shape[0],
                              None if op is None else _ptr(op, C.c_int64), _ptr(d, C.c_double))
        return d

    def ray_neumann(self, x, nu, tmax):
        x = np.ascontiguousarray(x, np.float64)
        nu = np.ascontiguousarray(nu, np.float64)
        tmax = np.ascontiguousarray(np.broadcast_to(tmax, (x.shape[0],)), np.float64)
        t = np.zeros(x.shape[0])
        pr = np.zeros(x.shape[0], np.int64)
        self._L.or_ray_neumann(self.h, _ptr(x, C.c_double), _ptr(nu, C.c_double),
                               _ptr(tmax, C.c_double), x.shape[0], _ptr(t, C.c_double),
                               _ptr(pr, C.c_int64))
        return t, pr


def estimates(res):
    """Per-point mean, standard error and count from accumulated sums."""
    n = res["count"].astype(np.float64)
    mean = res["sum"] / n
    var = np.maximum(res["sumsq"] / n - mean * mean, 0.0) * n / np.maximum(n - 1, 1)
    return mean, np.sqrt(var / n), n
