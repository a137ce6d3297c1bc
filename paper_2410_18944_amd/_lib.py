"""ctypes binding of ``libwost.so`` (the C ABI in include/wost.h).

Argument marshalling only: every step of the walk runs in the library's HIP
kernels.  The library must be built (``paper_2410_18944_amd.build``); there is
no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwost.so")

WOST_OK = 0
SAMPLING = {"uniform": 0, "mis_learned": 1, "mis_fixed": 2, "guided_only": 3}
FIELD = {"zero": 0, "const": 1, "exp_sin": 2, "re_z3": 3, "x2_minus_y2": 4, "r2": 5, "gauss_sum": 6}
MAX_GAUSS = 32


class wost_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("params", C.POINTER(C.c_float))]


class wost_problem(C.Structure):
    _fields_ = [("g", wost_field), ("h", wost_field), ("f", wost_field),
                ("eps", C.c_float), ("r_min", C.c_float),
                ("max_steps", C.c_int32), ("rr_start", C.c_int32), ("rr_q", C.c_float),
                ("sampling", C.c_int32), ("c_fixed", C.c_float), ("reflect", C.c_int32)]


class wost_build_opts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("brute_force", C.c_int32)]


class wost_records(C.Structure):
    _fields_ = [("data", C.c_void_p), ("capacity", C.c_int64), ("count", C.c_void_p)]


class wost_guide_config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("levels", C.c_int32), ("feats", C.c_int32), ("log2_table", C.c_int32),
                ("n_min", C.c_int32), ("n_max", C.c_int32), ("hidden", C.c_int32), ("n_hidden", C.c_int32),
                ("K", C.c_int32), ("aabb_lo", C.c_float * 3), ("aabb_hi", C.c_float * 3)]


class wost_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("e_mis", C.c_float)]


_P = C.c_void_p
_I = C.c_int
_I32 = C.c_int32
_I64 = C.c_int64
_U32 = C.c_uint32
_U64 = C.c_uint64
_F = C.c_float

# name -> (restype, argtypes); the Python names are the C names
SIGNATURES = {
    "wost_last_error": (C.c_char_p, []),
    "wost_build_bvh": (_I, [_I32, _P, _I64, _P, _I64, _P, C.POINTER(wost_build_opts), C.POINTER(_P)]),
    "wost_build_bvh_device_workspace": (_I, [_I32, _I64, _I64, C.POINTER(wost_build_opts), C.POINTER(_I64)]),
    "wost_build_bvh_device": (_I, [_I32, _P, _I64, _P, _I64, _P, C.POINTER(wost_build_opts), _P, _I64, _P,
                                   C.POINTER(_P)]),
    "wost_geom_device_bytes": (_I64, [_P]),
    "wost_geom_upload": (_I, [_P, _P, _I64, _P]),
    "wost_geom_info": (_I, [_P, C.POINTER(C.c_double)]),
    "wost_geom_prim_index": (_I64, [_P, _I32]),
    "wost_geom_free": (None, [_P]),
    "wost_query": (_I, [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "wost_neumann_sample": (_I, [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "wost_solve_workspace_bytes": (_I64, [_P, _I64, _I32]),
    "wost_solve": (_I, [_P, C.POINTER(wost_problem), _P, _I64, _I32, _U64, _U64, _P, _P, _P, _P, _P, _P,
                        C.POINTER(wost_records), _P, _I64, _P, _P]),
    "wost_solve_wavefront": (_I, [_P, C.POINTER(wost_problem), _P, _I64, _I32, _U64, _U64, _P, _P, _P, _P, _P,
                                  _P, C.POINTER(wost_records), _P, _I64, _P, _P]),
    "wost_solve_wavefront_workspace_bytes": (_I64, [_P, _I64, _I32]),
    "wost_set_wavefront_streams": (_I, [_I32]),
    "wost_lbvh_sizes": (_I, [_I32, _I64, _P, _P, _P]),
    "wost_geom_use_dirichlet_lbvh": (_I, [_P, _P, _I32, _P, _P, _I32, _I32]),
    "wost_lbvh_build": (_I, [_I32, _P, _I64, _I32, _P, _P, _P, _P, _P, _P, _I64, _P]),
    "wost_lbvh_closest": (_I, [_I32, _P, _I32, _P, _P, _I32, _I32, _P, _I64, _P, _P, _P]),
    "wost_set_launch": (_I, [_I32]),
    "wost_set_walk_pool": (_I, [_I32, _I32]),
    "wost_set_cost_counters": (_I, [_P]),
    "wost_guide_create": (_I, [C.POINTER(wost_guide_config), C.POINTER(_P)]),
    "wost_guide_param_count": (_I64, [_P]),
    "wost_guide_set_reflect": (_I, [_P, C.c_int32]),
    "wost_guide_get_reflect": (_I, [_P]),
    "wost_guide_shadow_bytes": (_I64, [_P]),
    "wost_guide_bind": (_I, [_P, _P, _P, _P, _P, _P]),
    "wost_guide_init": (_I, [_P, _U64, _P]),
    "wost_guide_sync_shadow": (_I, [_P, _P]),
    "wost_guide_infer": (_I, [_P, _P, _I64, _P, _P]),
    "wost_guide_sample": (_I, [_P, _I32, _F, _P, _P, _I64, _U64, _U32, _P, _P, _P]),
    "wost_guide_free": (None, [_P]),
    "wost_tail_pass": (_I, [_I32, C.POINTER(wost_records), _P, _I64, _P]),
    "wost_guide_loss_fwd": (_I, [_P, C.POINTER(wost_records), _I64, _I64, _F, _P, _P]),
    "wost_guide_loss_bwd": (_I, [_P, C.POINTER(wost_records), _I64, _I64, _F, _F, _P, _P, _P, _I64, _P]),
    "wost_guide_adam_step": (_I, [_P, C.POINTER(wost_adam), _P]),
    "wost_records_sample": (_I, [_I32, C.POINTER(wost_records), _U64, _I64, C.POINTER(wost_records), _P]),
    "wost_guide_train_step": (_I, [_P, C.POINTER(wost_records), _I64, _I64, C.POINTER(wost_adam), _P, _P, _I64, _P]),
    "wost_guide_train_step_noalloc": (_I, [_P, C.POINTER(wost_records), _I64, _I64, C.POINTER(wost_adam), _P, _P]),
    "wost_guide_train_workspace_bytes": (_I64, [_P, _I64]),
}

_lib = None


class WostError(RuntimeError):
    pass


def load():
    """Load libwost.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwost.so is not built: run paper_2410_18944_amd.build.build() "
                          "(the HIP library is required; there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    lib = load()
    return {name for name in SIGNATURES if getattr(lib, name, None) is not None}


def check(rc, what=""):
    if rc != WOST_OK:
        msg = load().wost_last_error()
        raise WostError("%s failed (%d): %s" % (what, rc, msg.decode() if msg else ""))
