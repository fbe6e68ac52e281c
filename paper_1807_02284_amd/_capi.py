"""ctypes binding of libcslbm.so (argument marshalling only).

Mirrors ``include/cslbm.h``.  Every compute step runs in the HIP kernels of
the library; this module only lays out the structs and forwards pointers.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcslbm.so")

OK = 0
ERR_ARG, ERR_SHAPE, ERR_UNSUPPORTED, ERR_HIP, ERR_NONFINITE = -1, -2, -3, -4, -5
F32, F16S = 0, 1
FLUID, SOLID, INLET, OUTFLOW, GHOST, NEUMANN, WALL, NEAR_WALL, NEAR_FLUID = 0, 1, 2, 3, 4, 5, 6, 8, 16
WALL_NORMAL_SHIFT = 5
GMAX_BUF = 1025

_vp = C.c_void_p


class CslbmParams(C.Structure):
    _fields_ = [
        ("nu", C.c_double),
        ("nu_hi", C.c_double * 4),
        ("a", C.c_double),
        ("b", C.c_double),
        ("g_max", C.c_double),
        ("adaptive", C.c_int32),
        ("grad_mode", C.c_int32),
        ("gmax_running", C.c_int32),
        ("tau_s", C.c_double),
        ("beta", C.c_double),
        ("s_ref", C.c_double),
        ("u_in", C.c_double * 3),
        ("s_in", C.c_double),
    ]


class CslbmLevel(C.Structure):
    _fields_ = [
        ("nx", C.c_int32),
        ("ny", C.c_int32),
        ("nz", C.c_int32),
        ("storage", C.c_int32),
        ("periodic", C.c_int32),
        ("reserved0", C.c_int32),
        ("plane", C.c_int64),
        ("f", _vp),
        ("f_next", _vp),
        ("g", _vp),
        ("g_next", _vp),
        ("flags", _vp),
        ("links", _vp),
        ("force", _vp),
        ("vel", _vp),
        ("vel_next", _vp),
        ("gmax_buf", _vp),
        ("brick_table", _vp),
        ("brick_origin", _vp),
        ("n_bricks", C.c_int32),
        ("wall_cells", C.c_int32),
        ("origin", C.c_double * 3),
        ("dx", C.c_double),
        ("p", CslbmParams),
    ]


MAX_SCALES = 8


class CslbmScale(C.Structure):
    _fields_ = [
        ("level", CslbmLevel),
        ("work_f", _vp * 2),
        ("work_g", _vp * 2),
        ("parent", C.c_int32),
        ("n_ghost", C.c_int32),
        ("ghost_cells", _vp),
        ("n_post", C.c_int32 * MAX_SCALES),
        ("post_cells", _vp * MAX_SCALES),
        ("n_ghost_xlo", C.c_int32),
        ("n_ghost_xhi", C.c_int32),
        ("ghost_xlo", C.c_int32),
        ("ghost_xhi", C.c_int32),
        ("stage", _vp),
        ("stage_bytes", C.c_int64),
        ("post_tiles", _vp * MAX_SCALES),
        ("n_post_tiles", C.c_int32 * MAX_SCALES),
        ("ghost_tiles", _vp),
        ("n_ghost_tiles", C.c_int32),
    ]


class CslbmHierarchy(C.Structure):
    _fields_ = [("n_scales", C.c_int32), ("reserved", C.c_int32),
                ("scales", C.POINTER(CslbmScale))]


class CslbmError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} failed with status {code}: {msg}")
        self.code = code


# name -> (restype, argtypes)
_SIGNATURES = {
    "cslbm_plane_stride": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "cslbm_level_bytes": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "cslbm_prepare_flags": (C.c_int, [C.POINTER(CslbmLevel), _vp]),
    "cslbm_init_equilibrium": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp]),
    "cslbm_set_populations": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, C.c_int32, _vp]),
    "cslbm_get_populations": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, C.c_int32, _vp]),
    "cslbm_copy_cells": (C.c_int, [C.POINTER(CslbmLevel), _vp, C.POINTER(CslbmLevel), _vp,
                                   C.c_int32, _vp]),
    "cslbm_step": (C.c_int, [C.POINTER(CslbmLevel), C.c_int32, _vp]),
    "cslbm_read_macro": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp]),
    "cslbm_vorticity": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp]),
    "cslbm_conserved_f64": (C.c_int, [C.POINTER(CslbmLevel), C.POINTER(C.c_double), _vp]),
    "cslbm_conserved_f64_noalloc": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp]),
    "cslbm_stage_bytes": (C.c_int64, [C.POINTER(CslbmLevel), C.POINTER(CslbmLevel), C.c_int32,
                                      C.c_int32]),
    "cslbm_check_finite": (C.c_int, [C.POINTER(CslbmLevel), C.POINTER(C.c_int64), _vp]),
    "cslbm_exchange": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp, C.c_double,
                                 C.POINTER(CslbmLevel), _vp, _vp, _vp, C.c_int32, _vp]),
    "cslbm_time_interp": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp, _vp, _vp,
                                    C.POINTER(C.c_double), C.c_double, _vp, _vp, _vp]),
    "cslbm_multiscale_step": (C.c_int, [C.POINTER(CslbmHierarchy), C.c_int32, _vp]),
    "cslbm_step_store": (C.c_int, [C.POINTER(CslbmLevel), C.c_int32, C.POINTER(_vp),
                                   C.POINTER(_vp), _vp]),
    "cslbm_adjoint_step": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp, _vp, _vp]),
    "cslbm_exchange_adjoint": (C.c_int, [C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp, C.c_double,
                                         C.POINTER(CslbmLevel), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         C.c_int32, _vp, C.c_int64, _vp]),
    "cslbm_exchange_adjoint_bytes": (C.c_int64, [C.POINTER(CslbmLevel), C.POINTER(CslbmLevel),
                                                 C.c_int32]),
    "cslbm_multiscale_adjoint_bytes": (C.c_int64, [C.POINTER(CslbmHierarchy)]),
    "cslbm_multiscale_adjoint_step": (C.c_int, [C.POINTER(CslbmHierarchy), C.POINTER(_vp),
                                                C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                                                _vp, C.c_int64, _vp]),
    "cslbm_abi_sizes": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "cslbm_last_error": (C.c_char_p, []),
}

_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> C.CDLL:
    """Load libcslbm.so; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_1807_02284_amd/build.py` first (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    pb, lb, sb = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    lib.cslbm_abi_sizes(C.byref(pb), C.byref(lb), C.byref(sb))
    want = (C.sizeof(CslbmParams), C.sizeof(CslbmLevel), C.sizeof(CslbmScale))
    if (pb.value, lb.value, sb.value) != want:
        raise RuntimeError(
            f"struct layout mismatch: library has cslbm_params={pb.value} B, cslbm_level="
            f"{lb.value} B, cslbm_scale={sb.value} B; binding has {want[0]} B, {want[1]} B, "
            f"{want[2]} B")
    _lib = lib
    return lib


def call(name: str, *args) -> int:
    """Call an int-returning entry point and raise CslbmError on failure."""
    lib = load()
    rc = getattr(lib, name)(*args)
    if rc < 0:
        msg = lib.cslbm_last_error().decode(errors="replace")
        raise CslbmError(rc, name, msg)
    return rc


def declared_symbols(header: str) -> list[str]:
    """Names of the functions declared in a C header (cslbm_* prototypes)."""
    import re
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cslbm_[a-z0-9_]+)\s*\(", text)))
