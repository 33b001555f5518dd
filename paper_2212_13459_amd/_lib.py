"""ctypes declarations for libnst.so (include/nst.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_size_t, c_uint, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnst.so")

NST_MAX_CONV = 16
NST_MAX_STYLE = 8
NST_FP32, NST_BF16 = 0, 1
NST_STEP1, NST_STEP2, NST_BOTH, NST_STRICT_HALO, NST_CHECK_FINITE, NST_RESIDENT = 1, 2, 3, 4, 8, 16

STATUS = {0: "NST_OK", -1: "NST_EINVAL", -2: "NST_ESHAPE", -3: "NST_EHALO", -4: "NST_ENOMEM",
          -5: "NST_EHIP", -6: "NST_ECAPACITY", -7: "NST_EWORKSPACE", -8: "NST_ENONFINITE"}


class NetDesc(ctypes.Structure):
    _fields_ = [("n_conv", c_int), ("c_in", c_int * NST_MAX_CONV), ("c_out", c_int * NST_MAX_CONV),
                ("pool_after", c_uint), ("n_style", c_int), ("style_conv", c_int * NST_MAX_STYLE),
                ("content_conv", c_int), ("pool_avg", c_uint)]


class Tile(ctypes.Structure):
    _fields_ = [("by0", c_int), ("by1", c_int), ("bx0", c_int), ("bx1", c_int),
                ("ey0", c_int), ("ey1", c_int), ("ex0", c_int), ("ex1", c_int),
                ("own", (c_int * 4) * NST_MAX_CONV)]


class MeanStd(ctypes.Structure):
    _fields_ = [("w_mean", POINTER(c_double)), ("w_std", POINTER(c_double)), ("target_means", c_void_p),
                ("means_x", c_void_p)]


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 160), ("launches", c_int), ("ms", c_double), ("flops", c_double),
                ("bytes", c_double)]


class NstError(RuntimeError):
    def __init__(self, fn, status, lib=None):
        msg = STATUS.get(status, str(status))
        if lib is not None:
            msg += ": " + lib.nst_strerror(status).decode()
        super().__init__(f"{fn} failed with {msg}")
        self.status = status


_lib = None

SIGNATURES = {
    "nst_abi_version": (c_int, []),
    "nst_strerror": (ctypes.c_char_p, [c_int]),
    "nst_net_vgg19": (c_int, [POINTER(NetDesc), c_int, c_int]),
    "nst_min_halo": (c_int, [POINTER(NetDesc)]),
    "nst_plan": (c_int, [POINTER(NetDesc), c_int, c_int, c_int, c_int, POINTER(Tile), c_int, POINTER(c_int)]),
    "nst_workspace_bytes": (c_int, [POINTER(NetDesc), c_int, c_int, c_int, c_int, c_int, c_int, POINTER(c_size_t)]),
    "nst_create": (c_int, [POINTER(NetDesc), POINTER(POINTER(c_float)), POINTER(POINTER(c_float)), c_int,
                           POINTER(c_void_p)]),
    "nst_destroy": (None, [c_void_p]),
    "nst_style_grams": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_size_t,
                                c_void_p]),
    "nst_layer_feats": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p,
                                c_size_t, c_void_p]),
    "nst_content_feats": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_size_t,
                                  c_void_p]),
    "nst_profile": (c_int, [c_void_p, c_int]),
    "nst_profile_read": (c_int, [c_void_p, POINTER(KStat), c_int, POINTER(c_int)]),
    "nst_loss_grad": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, POINTER(c_double), c_double,
                              c_int, c_int, c_int, c_void_p, POINTER(c_double), c_void_p, c_void_p, c_size_t,
                              c_void_p]),
    "nst_scratch_bytes": (c_size_t, []),
    "nst_loss_grad_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, POINTER(c_double),
                                      c_double, c_int, c_int, c_int, c_void_p, POINTER(c_double), c_void_p,
                                      c_void_p]),
    "nst_style_stats": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                c_size_t, c_void_p]),
    "nst_loss_grad_ms": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, POINTER(c_double),
                                 c_double, POINTER(MeanStd), c_int, c_int, c_int, c_void_p, POINTER(c_double),
                                 c_void_p, c_void_p, c_size_t, c_void_p]),
}


def lib():
    """Load libnst.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_13459_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn, status):
    if status != 0:
        raise NstError(fn, status, _lib)
