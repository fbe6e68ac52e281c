"""Host-side checks of the C ABI: the library loads without a GPU, exports
every function the header declares, agrees with the binding on struct
layout, and rejects bad arguments before any launch."""
import ctypes as C
import os

import pytest

from paper_1807_02284_amd import _capi
from paper_1807_02284_amd.level import Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


@pytest.fixture(scope="module")
def lib():
    return _capi.load()


def test_every_declared_function_is_exported(lib):
    names = []
    for h in HEADERS:
        names += _capi.declared_symbols(h)
    assert "cslbm_step" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    names = set()
    for h in HEADERS:
        names |= set(_capi.declared_symbols(h))
    assert names == set(_capi._SIGNATURES), names ^ set(_capi._SIGNATURES)


def test_plane_stride_and_level_bytes(lib):
    p = lib.cslbm_plane_stride(256, 256, 256)
    assert p >= 256 ** 3 and p % 256 == 0 and (p // 256) % 2 == 1
    assert lib.cslbm_level_bytes(256, 256, 256, _capi.F32, 0) == 27 * p * 4
    assert lib.cslbm_level_bytes(256, 256, 256, _capi.F16S, 1) == 27 * p * 2 + 7 * p * 4
    assert lib.cslbm_plane_stride(0, 4, 4) == _capi.ERR_SHAPE
    assert lib.cslbm_level_bytes(4, 4, 4, 7, 0) == _capi.ERR_UNSUPPORTED


def make_level(**kw):
    L = _capi.CslbmLevel()
    L.nx, L.ny, L.nz = 8, 8, 8
    L.storage = _capi.F32
    L.periodic = 7
    L.plane = 1024
    L.f = 0x1000          # never dereferenced: validation fails before any launch
    L.f_next = 0x2000
    L.p = Params(nu=0.01).to_c()
    for k, v in kw.items():
        if k.startswith("p_"):
            setattr(L.p, k[2:], v)
        else:
            setattr(L, k, v)
    return L


@pytest.mark.parametrize("kw,code,needle", [
    (dict(nx=0), _capi.ERR_SHAPE, "positive"),
    (dict(plane=100), _capi.ERR_SHAPE, "plane stride"),
    (dict(storage=5), _capi.ERR_UNSUPPORTED, "storage"),
    (dict(f=None), _capi.ERR_ARG, "f is NULL"),
    (dict(f_next=0x1000), _capi.ERR_ARG, "alias"),
    (dict(periodic=5), _capi.ERR_ARG, "flags"),
    (dict(p_nu=0.0), _capi.ERR_ARG, "viscosity"),
    (dict(p_nu=-1.0), _capi.ERR_ARG, "viscosity"),
    (dict(p_g_max=0.0), _capi.ERR_ARG, "g_max"),
    (dict(p_a=-6.0), _capi.ERR_ARG, "adaptive factor"),
    (dict(g=0x3000), _capi.ERR_ARG, "g_next"),
])
def test_step_rejects_bad_arguments_before_launch(lib, kw, code, needle):
    L = make_level(**kw)
    rc = lib.cslbm_step(C.byref(L), 1, None)
    assert rc == code
    assert needle in lib.cslbm_last_error().decode()


def test_negative_step_count_and_null_level(lib):
    L = make_level()
    assert lib.cslbm_step(C.byref(L), -1, None) == _capi.ERR_ARG
    assert lib.cslbm_step(None, 1, None) == _capi.ERR_ARG
    assert lib.cslbm_conserved_f64(C.byref(L), None, None) == _capi.ERR_ARG
    assert lib.cslbm_conserved_f64_noalloc(C.byref(L), None, None) == _capi.ERR_ARG
    assert lib.cslbm_conserved_f64_noalloc(None, 0x5000, None) == _capi.ERR_ARG
    assert lib.cslbm_check_finite(C.byref(L), None, None) == _capi.ERR_ARG


def test_scalar_relaxation_time_checked(lib):
    L = make_level(g=0x3000, g_next=0x4000, p_tau_s=0.5)
    assert lib.cslbm_step(C.byref(L), 1, None) == _capi.ERR_ARG
    assert "tau_s" in lib.cslbm_last_error().decode()


def test_stage_bytes_of_a_padded_box_inside_its_parent(lib):
    """x-face staging work space: two planes x 2 time levels x (27 float
    planes + 7 scalar planes) over a sub-box of at most 4 parent columns and
    the rows the plane's stencils reach; 0 when a plane's stencils leave the
    parent (here the padding column beyond the shell), negative for a bad
    level."""
    P = make_level(periodic=0, flags=0x9000)
    P.nx, P.ny, P.nz = 512, 256, 256
    P.plane = lib.cslbm_plane_stride(512, 256, 256)
    P.dx = 1.0
    L = make_level(periodic=0, flags=0x9100, g=0x3000, g_next=0x4000)
    L.nx, L.ny, L.nz = 768, 116, 116          # 759 cells padded to 768 along x
    L.plane = lib.cslbm_plane_stride(768, 116, 116)
    L.dx = 1 / 1.5
    L.origin[0], L.origin[1], L.origin[2] = 3.0, 89.0, 89.0
    n = lib.cslbm_stage_bytes(C.byref(P), C.byref(L), 0, 758)
    rows = 80 * 80                            # parent rows 88..167 along y and z
    per_face = 2 * (27 * 4 + 7 * 4) * 4 * rows
    assert n == per_face * 2
    assert lib.cslbm_stage_bytes(C.byref(P), C.byref(L), 0, 767) == 0
    assert lib.cslbm_stage_bytes(C.byref(P), None, 0, 758) < 0
