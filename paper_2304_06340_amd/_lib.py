"""ctypes declarations of the C ABI in include/hsd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
import threading

from ._build import LIB, TEST_LIB

HSD_OK, HSD_PENDING = 0, 1
HSD_EINVAL, HSD_ENOMEM, HSD_EDEVICE, HSD_EAGAIN, HSD_ECANCELED, HSD_ENOTFOUND = -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
FORM_FP64, FORM_MIXED = 0, 1
METHOD_DIRECT, METHOD_NUFFT3 = 0, 1
RULE_SPHERICAL_PRODUCT, RULE_EXPLICIT, RULE_CUBE_TRAPEZOID = 0, 1, 2
TRI_DUNAVANT7, TRI_GL8X8 = 0, 1

STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE",
                -4: "EAGAIN", -5: "ECANCELED", -6: "ENOTFOUND"}

dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int32)


class RuleDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("r_max", C.c_double), ("n_panels", C.c_int32),
                ("n_per_panel", C.c_int32), ("n_cos", C.c_int32), ("n_phi", C.c_int32),
                ("nodes", dp), ("weights", dp), ("n_nodes", C.c_int64),
                ("xi_max", C.c_double), ("M", C.c_int32)]


class SurfaceDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_u", C.c_int32), ("n_v", C.c_int32), ("a", C.c_double),
                ("b", C.c_double), ("c", C.c_double), ("center", C.c_double * 3), ("reserved", C.c_int32 * 4)]


SURFACE_ELLIPSOID, SURFACE_TORUS = 0, 1


class Params(C.Structure):
    _fields_ = [("s", C.c_double), ("form", C.c_int32), ("method", C.c_int32),
                ("taylor_tau", C.c_double), ("tri_rule", C.c_int32), ("nufft_tol", C.c_double),
                ("nufft_width", C.c_int32), ("nufft_sigma", C.c_double), ("k_splits", C.c_int32),
                ("reserved0", C.c_int32), ("freq_unit", C.c_double), ("reserved", C.c_int32 * 4)]


class Result(C.Structure):
    _fields_ = [("d2", C.c_double), ("rel_err_stated", C.c_double), ("pairs", C.c_double),
                ("device_ms", C.c_double), ("transform_ms", C.c_double), ("status", C.c_int32),
                ("reserved", C.c_int32)]


class ServerCfg(C.Structure):
    _fields_ = [("slots", C.c_int32), ("queue_capacity", C.c_int32),
                ("hbm_budget_bytes", C.c_size_t), ("chunk_pairs", C.c_int64),
                ("reserved", C.c_int32 * 8)]


class Request(C.Structure):
    _fields_ = [("verts", dp), ("nv", C.c_int64), ("tris", ip), ("nt", C.c_int64),
                ("verts2", dp), ("nv2", C.c_int64), ("tris2", ip), ("nt2", C.c_int64),
                ("rule", C.c_void_p), ("params", Params), ("tag", C.c_int64)]


class RequestTimes(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("admitted_s", C.c_double),
                ("finished_s", C.c_double), ("footprint", C.c_int64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "hsd_version": (C.c_char_p, []),
    "hsd_last_error": (C.c_char_p, []),
    "hsd_params_default": (None, [C.POINTER(Params)]),
    "hsd_init": (C.c_int32, [C.c_int, C.c_size_t, C.POINTER(C.c_void_p)]),
    "hsd_ctx_set_stream": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "hsd_ctx_bytes_in_use": (C.c_size_t, [C.c_void_p]),
    "hsd_finalize": (None, [C.c_void_p]),
    "hsd_create_mesh": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                    C.c_int32, C.POINTER(C.c_void_p)]),
    "hsd_create_point_measure": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                             C.POINTER(C.c_void_p)]),
    "hsd_create_surface_measure": (C.c_int32, [C.c_void_p, C.POINTER(SurfaceDesc), C.POINTER(C.c_void_p)]),
    "hsd_mesh_num_triangles": (C.c_int64, [C.c_void_p]),
    "hsd_mesh_num_vertices": (C.c_int64, [C.c_void_p]),
    "hsd_mesh_destroy": (None, [C.c_void_p]),
    "hsd_freq_rule": (C.c_int32, [C.c_void_p, C.POINTER(RuleDesc), C.POINTER(C.c_void_p)]),
    "hsd_rule_num_nodes": (C.c_int64, [C.c_void_p]),
    "hsd_rule_nodes": (C.c_int32, [C.c_void_p, dp, dp]),
    "hsd_rule_destroy": (None, [C.c_void_p]),
    "hsd_distance": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.POINTER(Params), C.POINTER(Result)]),
    "hsd_ctx_set_stage_timing": (C.c_int32, [C.c_void_p, C.c_int32]),
    "hsd_nufft_stage_stats": (C.c_int32, [C.c_void_p, dp, dp]),
    "hsd_distance_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.POINTER(Params), C.POINTER(Result)]),
    "hsd_distance_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(Params), C.c_void_p, C.c_int32, C.POINTER(Result)]),
    "hsd_transform": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                  C.POINTER(Params), C.c_void_p, C.c_int32]),
    "hsd_transform_rule": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Params),
                                       C.c_void_p, C.c_int32]),
    "hsd_server_create": (C.c_int32, [C.c_void_p, C.POINTER(ServerCfg), C.POINTER(C.c_void_p)]),
    "hsd_submit": (C.c_int32, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "hsd_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(Result), C.POINTER(RequestTimes)]),
    "hsd_wait": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_double, C.POINTER(Result),
                             C.POINTER(RequestTimes)]),
    "hsd_cancel": (C.c_int32, [C.c_void_p, C.c_uint64]),
    "hsd_release": (C.c_int32, [C.c_void_p, C.c_uint64]),
    "hsd_server_destroy": (None, [C.c_void_p]),
}

_libs = {}
_lock = threading.Lock()


def _open(p: str):
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: the HIP library has not been built "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def load(path: str | None = None):
    """Load libhsd.so; raises if it has not been built (there is no fallback)."""
    p = path or LIB
    with _lock:
        if p not in _libs:
            _libs[p] = _open(p)
    return _libs[p]


def load_test_hooks():
    """libhsd_testhooks.so: the same library built with the test hooks (CPU
    runs of the lane bodies, the FFT on its own, the simulated serving
    executor).  For tests only; objects created through one library must
    not be passed to the other."""
    return load(TEST_LIB)


def exported_symbols() -> list[str]:
    return list(SIGNATURES)
