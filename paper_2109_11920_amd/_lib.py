"""ctypes declarations of the libboac C ABI (include/boac.h). Loading fails loudly if the library is
not built: there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libboac.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "boac.h")

c_int32 = ctypes.c_int32
c_float = ctypes.c_float
c_void_p = ctypes.c_void_p


class BoacGeom(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_angles", c_int32), ("n_bins", c_int32), ("n_samples", c_int32),
                ("pixel_cm", c_float)]


class BoacSlice(ctypes.Structure):
    _fields_ = [("geom", BoacGeom), ("d_meas", c_void_p), ("d_cand", c_void_p), ("C", c_int32),
                ("d_obj", c_void_p), ("d_grad", c_void_p), ("d_status", c_void_p)]


STATUS_NAMES = {0: "BOAC_OK", 1: "BOAC_EINVAL", 2: "BOAC_ESHAPE", 3: "BOAC_ENOMEM", 4: "BOAC_EDEVICE",
                5: "BOAC_ETIMEOUT", 6: "BOAC_ENOTSUP"}

KERNEL_KINDS = {"raster": 0, "att": 1, "fwd": 2, "back": 3, "reduce": 4, "adj_ray": 5, "adj_pix": 6, "other": 7,
                "gp": 8}


class BoacGpInfo(ctypes.Structure):
    _fields_ = [("n", c_int32), ("d", c_int32), ("length", ctypes.c_double), ("amp", ctypes.c_double),
                ("noise", ctypes.c_double), ("m0", ctypes.c_double), ("s", ctypes.c_double),
                ("lml", ctypes.c_double)]

_P = c_void_p
_SIGNATURES = {
    "boac_version": (c_int32, []),
    "boac_ctx_create": (c_int32, [c_int32, ctypes.c_char_p, ctypes.POINTER(c_void_p)]),
    "boac_ctx_destroy": (None, [_P]),
    "boac_last_error": (ctypes.c_char_p, []),
    "boac_rasterize_mu": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, c_int32, c_float, _P, _P]),
    "boac_project": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, _P, _P]),
    "boac_backproject": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, _P, _P]),
    "boac_mlem": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, c_int32, _P, _P]),
    "boac_objective": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, c_float, c_int32, _P, _P, _P,
                                 _P]),
    "boac_objective_noalloc": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, c_float, c_int32, _P, _P,
                                         _P, _P]),
    "boac_objective_grad": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, c_float, c_int32, c_int32,
                                      _P, _P, _P, _P]),
    "boac_objective_grad_ex": (c_int32, [_P, ctypes.POINTER(BoacGeom), _P, _P, c_int32, c_float, c_int32, c_int32,
                                         c_int32, _P, _P, _P, _P]),
    "boac_evaluate_batch": (c_int32, [_P, ctypes.POINTER(BoacSlice), c_int32, c_float, c_int32, c_int32, _P]),
    "boac_gp_fit": (c_int32, [_P, _P, c_int32, c_int32, _P, c_int32, c_int32, ctypes.c_double, _P, _P,
                              ctypes.POINTER(BoacGpInfo)]),
    "boac_gp_ei": (c_int32, [_P, ctypes.POINTER(BoacGpInfo), _P, _P, _P, _P, c_int32, ctypes.c_double,
                             ctypes.c_double, _P, _P, _P, _P]),
    "boac_gp_chaos_local": (c_int32, [_P, ctypes.POINTER(BoacGpInfo), _P, _P, _P, ctypes.c_double, ctypes.c_double,
                                      _P, c_int32, _P, _P, c_int32, ctypes.c_double, ctypes.c_double, c_int32, _P,
                                      _P, _P]),
    "boac_gp_chaos_search": (c_int32, [_P, ctypes.POINTER(BoacGpInfo), _P, _P, _P, ctypes.c_double, ctypes.c_double,
                                       _P, c_int32, c_int32, c_int32, c_int32, c_int32, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, c_int32, _P, c_int32, _P,
                                       ctypes.POINTER(c_int32), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64), _P]),
    "boac_ctx_set_profiling": (c_int32, [_P, c_int32]),
    "boac_ctx_kernel_stats": (c_int32, [_P, c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "boac_ctx_reset_stats": (c_int32, [_P]),
    "boac_ctx_set_batch_mode": (c_int32, [_P, c_int32, ctypes.c_int64]),
    "boac_ctx_graph_stats": (c_int32, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


class BoacError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


def header_functions(path: str = HEADER_PATH):
    """Names of every function declared in include/boac.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(boac_[a-z_]+)\s*\(", text)))


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libboac.so is not built ({LIB_PATH}); run "
                          f"`python -m paper_2109_11920_amd.build` or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != 0:
        msg = load().boac_last_error()
        raise BoacError(code, msg.decode() if msg else "")
