"""ctypes declarations mirroring include/tpfa.h, and the loader of libtpfa.so.

The library is loaded from this package directory only; a missing or
unloadable library raises immediately (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpfa.so")

TPFA_OK = 0
TPFA_ERR_NULL = -1
TPFA_ERR_SHAPE = -2
TPFA_ERR_PARAM = -3
TPFA_ERR_UNSUPPORTED = -4
TPFA_ERR_HIP = -5
TPFA_ERR_TILE = -6

TPFA_FP64 = 0
TPFA_FP32 = 1
# tpfa_op_t
TPFA_OP_RESIDUAL, TPFA_OP_JACOBIAN, TPFA_OP_VJP, TPFA_OP_RESIDUAL10 = 0, 1, 2, 3
TPFA_OP_RESIDUAL_BE, TPFA_OP_JACOBIAN_BE, TPFA_OP_JVP, TPFA_OP_JVP_BE = 4, 5, 6, 7
TPFA_BATCH_RESIDUAL = 0
TPFA_BATCH_JACOBIAN = 1
TPFA_LAUNCH_XCD_REMAP = 1
TPFA_LAUNCH_Y_FAST = 2
TPFA_LAUNCH_PAD_WRITES = 4
TPFA_LAUNCH_SLICED = 8
TPFA_TILE_FIT = 10
TPFA_SCHEDULE_PERSISTENT = 0
TPFA_SCHEDULE_GROUPED = 1


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("gk", C.c_double), ("ldx", C.c_int64)]


class Fluid(C.Structure):
    _fields_ = [("rho0", C.c_double), ("cf", C.c_double), ("p0", C.c_double),
                ("mu", C.c_double)]


class Rock(C.Structure):
    _fields_ = [("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p),
                ("ry", C.c_double), ("rz", C.c_double), ("seal", C.c_void_p),
                ("tx", C.c_void_p), ("ty", C.c_void_p), ("tz", C.c_void_p)]


class State(C.Structure):
    _fields_ = [("p", C.c_void_p), ("pref", C.c_void_p)]


class Accum(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("p_prev", C.c_void_p), ("dt", C.c_double),
                ("cr", C.c_double)]


class Launch(C.Structure):
    _fields_ = [("tile", C.c_int), ("kz_chunk", C.c_int), ("flags", C.c_int),
                ("y_begin", C.c_int64), ("y_end", C.c_int64)]


class Model(C.Structure):
    _fields_ = [("grid", Grid), ("fluid", Fluid), ("rock", Rock), ("state", State),
                ("r", C.c_void_p), ("J", C.c_void_p), ("launch", Launch)]


P = C.POINTER
vp = C.c_void_p

# name -> (restype, argtypes); every symbol declared in include/tpfa.h
SIGNATURES = {
    "tpfa_residual": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), C.c_int, vp, P(Launch), vp]),
    "tpfa_jacobian": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), C.c_int, vp, vp, P(Launch),
                                vp]),
    "tpfa_residual_vjp": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), C.c_int, vp, vp, vp,
                                    P(Launch), vp]),
    "tpfa_residual_and_vjp": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), C.c_int, vp, vp,
                                        vp, vp, P(Launch), vp]),
    "tpfa_residual_be": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), P(Accum), C.c_int,
                                   vp, P(Launch), vp]),
    "tpfa_jacobian_be": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), P(Accum), C.c_int,
                                   vp, vp, P(Launch), vp]),
    "tpfa_jvp": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), P(Accum), C.c_int, vp, vp,
                           vp, P(Launch), vp]),
    "tpfa_residual_vjp_trans": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), C.c_int, vp, vp,
                                          vp, P(Launch), vp]),
    "tpfa_residual10": (C.c_int, [P(Grid), P(Fluid), P(Rock), P(State), C.c_int, vp, vp, vp,
                                  P(Launch), vp]),
    "tpfa_hydrostatic": (C.c_int, [P(Grid), P(Fluid), C.c_double, vp, vp]),
    "tpfa_offset_pressure": (C.c_int, [P(Grid), vp, vp, vp, vp]),
    "tpfa_batch_create": (C.c_int, [P(Model), C.c_int, C.c_int, C.c_int, P(vp), vp]),
    "tpfa_batch_run": (C.c_int, [vp, vp]),
    "tpfa_batch_run_eager": (C.c_int, [vp, vp]),
    "tpfa_batch_info": (C.c_int, [vp, P(C.c_int64), P(C.c_int)]),
    "tpfa_batch_set_schedule": (C.c_int, [vp, C.c_int]),
    "tpfa_batch_destroy": (None, [vp]),
    "tpfa_num_tiles": (C.c_int, []),
    "tpfa_tile_shape": (C.c_int, [C.c_int, P(C.c_int), P(C.c_int), P(C.c_int)]),
    "tpfa_fit_tile_shape": (C.c_int, [C.c_int64, C.c_int64, P(C.c_int), P(C.c_int)]),
    "tpfa_strerror": (C.c_char_p, [C.c_int]),
    "tpfa_last_error": (C.c_char_p, []),
    "tpfa_version": (C.c_int, []),
    "tpfa_resolve_launch": (C.c_int, [P(Grid), C.c_int, C.c_int, P(Rock), P(Launch), P(Launch)]),
    "tpfa_stream_probe": (C.c_int, [P(Grid), C.c_int, vp, vp, vp, vp, vp]),
    "tpfa_stream_probe_sliced": (C.c_int, [P(Grid), C.c_int, vp, vp, vp, vp, vp]),
    "tpfa_ensemble_run_noalloc": (C.c_int, [P(Model), C.c_int, C.c_int, C.c_int, vp]),
}

_lib = None


# major version of the struct layouts below (TPFA_VERSION / 10000 in include/tpfa.h)
ABI_MAJOR = 2


def load():
    """Load libtpfa.so from the package directory (raises if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2304_11274_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.tpfa_version() // 10000 != ABI_MAJOR:
            raise RuntimeError(
                f"{LIB_PATH} has version {lib.tpfa_version()}, this binding's structs are "
                f"those of major version {ABI_MAJOR}: rebuild it with "
                "`python -m paper_2304_11274_amd.build`")
        _lib = lib
    return _lib


class TpfaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tpfa error {code}: {msg}")
        self.code = code


def check(rc: int, lib=None):
    if rc != TPFA_OK:
        lib = lib or load()
        raise TpfaError(rc, (lib.tpfa_last_error() or b"").decode() or
                        lib.tpfa_strerror(rc).decode())
    return rc
