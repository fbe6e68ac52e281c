"""Host-side argument checks of the multi-scale, copy, adjoint and
gradient-mode entry points: every case here fails validation and returns
its error code and message before any launch (no GPU needed)."""
import ctypes as C

import pytest

from paper_1807_02284_amd import _capi
from test_capi_abi import make_level


@pytest.fixture(scope="module")
def lib():
    return _capi.load()


def err(lib):
    return lib.cslbm_last_error().decode()


def test_exchange_argument_checks(lib):
    src, dst = make_level(dx=1.0), make_level(dx=0.5)
    cells = (C.c_int32 * 4)(0, 1, 2, 3)
    ex = lib.cslbm_exchange
    assert ex(C.byref(src), None, None, None, None, 0.0, C.byref(dst), 0x5000, None, cells, 4, None) == _capi.ERR_ARG
    assert "NULL" in err(lib)
    assert ex(C.byref(src), 0x1000, None, None, None, 0.0, C.byref(dst), 0x5000, None, None, 4, None) == _capi.ERR_ARG
    assert "cell list" in err(lib)
    assert ex(C.byref(src), 0x1000, None, None, None, 1.5, C.byref(dst), 0x5000, None, cells, 4, None) == _capi.ERR_ARG
    assert "time weight" in err(lib)
    bad = make_level(dx=0.0)
    assert ex(C.byref(src), 0x1000, None, None, None, 0.0, C.byref(bad), 0x5000, None, cells, 4, None) == _capi.ERR_ARG
    assert "spacing" in err(lib)
    singular = make_level(dx=1.0, p_nu=1.0 / 6.0)   # tau = 1: (I - S)^-1 is singular
    assert ex(C.byref(singular), 0x1000, None, None, None, 0.0, C.byref(dst), 0x5000, None, cells, 4,
              None) == _capi.ERR_ARG
    assert "singular" in err(lib)


def test_time_interp_argument_checks(lib):
    L = make_level()
    t = (C.c_double * 3)(0.0, 0.5, 0.5)
    ti = lib.cslbm_time_interp
    assert ti(C.byref(L), 0x1000, 0x2000, 0x3000, None, None, None, t, 1.0, 0x4000, None, None) == _capi.ERR_ARG
    assert "distinct" in err(lib)
    t2 = (C.c_double * 3)(0.0, 0.5, 1.0)
    assert ti(C.byref(L), 0x1000, None, 0x3000, None, None, None, t2, 1.0, 0x4000, None, None) == _capi.ERR_ARG


def hierarchy_of(levels, parents, **per_scale):
    scales = (_capi.CslbmScale * len(levels))()
    for i, (L, p) in enumerate(zip(levels, parents)):
        scales[i].level = L
        scales[i].parent = p
        scales[i].work_f = (C.c_void_p * 2)(0x7000 + i, 0x8000 + i)
        for k, v in per_scale.get(i, {}).items():
            setattr(scales[i], k, v)
    return _capi.CslbmHierarchy(len(levels), 0, C.cast(scales, C.POINTER(_capi.CslbmScale))), scales


def test_multiscale_step_argument_checks(lib):
    ms = lib.cslbm_multiscale_step
    assert ms(None, 1, None) == _capi.ERR_ARG
    L0 = make_level(dx=1.0)
    H, keep = hierarchy_of([L0], [-1])
    assert ms(C.byref(H), -1, None) == _capi.ERR_ARG
    H0 = _capi.CslbmHierarchy(0, 0, C.cast(keep, C.POINTER(_capi.CslbmScale)))
    assert ms(C.byref(H0), 1, None) == _capi.ERR_ARG
    # a finer scale without flags
    L1 = make_level(dx=0.5, periodic=0)
    H, keep = hierarchy_of([L0, L1], [-1, 0])
    assert ms(C.byref(H), 1, None) < 0
    # a finer scale whose parent index is not smaller than its own
    L1 = make_level(dx=0.5, flags=0x9000, periodic=0)
    H, keep = hierarchy_of([L0, L1], [-1, 1])
    assert ms(C.byref(H), 1, None) == _capi.ERR_ARG
    assert "parent" in err(lib)
    # a far-field scale posting onto anything but its parent's shell
    far = make_level(dx=2.0, flags=0x9000, periodic=0)
    H, keep = hierarchy_of([L0, far], [-1, 0])
    keep[1].n_post[1] = 3
    keep[1].post_cells[1] = 0xA000
    assert ms(C.byref(H), 1, None) == _capi.ERR_ARG
    assert "far-field" in err(lib)
    # a far-field scale whose parent is not the reference scale
    L1 = make_level(dx=0.5, flags=0x9000, periodic=0)
    H, keep = hierarchy_of([L0, L1, far], [-1, 0, 1])
    assert ms(C.byref(H), 1, None) == _capi.ERR_ARG
    assert "reference scale" in err(lib)
    # a finer scale posting onto a later finer scale
    L2 = make_level(dx=0.25, flags=0x9000, periodic=0)
    H, keep = hierarchy_of([L0, L1, L2], [-1, 0, 1])
    keep[1].n_post[2] = 3
    keep[1].post_cells[2] = 0xA000
    assert ms(C.byref(H), 1, None) == _capi.ERR_ARG
    assert "larger scales" in err(lib)
    # run offsets of a post-mapping list: more runs than entries, a negative
    # count, or a count without offsets
    H, keep = hierarchy_of([L0, L1], [-1, 0])
    keep[1].n_post[0] = 3
    keep[1].post_cells[0] = 0xA000
    for n_runs, ptr in ((4, 0xB000), (-1, 0xB000), (2, None)):
        keep[1].n_post_tiles[0] = n_runs
        keep[1].post_tiles[0] = ptr
        assert ms(C.byref(H), 1, None) == _capi.ERR_ARG
        assert "run offsets" in err(lib)
    # run offsets of a ghost list: more runs than ghosts, a negative count,
    # or a count without offsets
    H, keep = hierarchy_of([L0, L1], [-1, 0])
    keep[1].n_ghost = 3
    keep[1].ghost_cells = 0xA000
    for n_runs, ptr in ((4, 0xB000), (-1, 0xB000), (2, None)):
        keep[1].n_ghost_tiles = n_runs
        keep[1].ghost_tiles = ptr
        assert ms(C.byref(H), 1, None) == _capi.ERR_ARG
        assert "ghost list" in err(lib)
    # the gradient mode is single-level only
    Lg = make_level(p_grad_mode=1)
    H, keep = hierarchy_of([Lg], [-1])
    assert ms(C.byref(H), 1, None) == _capi.ERR_UNSUPPORTED


def test_copy_cells_argument_checks(lib):
    a, b = make_level(), make_level(f=0x6000)
    cells = (C.c_int32 * 2)(0, 1)
    cc = lib.cslbm_copy_cells
    half = make_level(storage=_capi.F16S, f=0x6000)
    assert cc(C.byref(a), cells, C.byref(half), cells, 2, None) == _capi.ERR_UNSUPPORTED
    assert cc(C.byref(a), None, C.byref(b), cells, 2, None) == _capi.ERR_ARG
    assert cc(C.byref(a), cells, C.byref(make_level()), cells, 2, None) == _capi.ERR_ARG
    assert "alias" in err(lib)
    sc = make_level(f=0x6000, g=0x3000, g_next=0x4000)
    assert cc(C.byref(a), cells, C.byref(sc), cells, 2, None) == _capi.ERR_ARG
    assert cc(C.byref(a), cells, C.byref(b), cells, 0, None) == _capi.OK   # nothing to do


def test_adjoint_and_step_store_argument_checks(lib):
    L = make_level()
    adj = lib.cslbm_adjoint_step
    assert adj(C.byref(L), None, None, 0x5000, None, None, None) == _capi.ERR_ARG
    assert adj(C.byref(L), 0x5000, None, 0x5000, None, None, None) == _capi.ERR_ARG
    assert "alias" in err(lib)
    open_box = make_level(periodic=3)                # no flags: only fully periodic boxes
    assert adj(C.byref(open_box), 0x5000, None, 0x6000, None, None, None) < 0
    grad = make_level(p_grad_mode=1)
    assert adj(C.byref(grad), 0x5000, None, 0x6000, None, None, None) == _capi.ERR_UNSUPPORTED
    scalar = make_level(g=0x3000, g_next=0x4000, p_tau_s=0.6)
    assert adj(C.byref(scalar), 0x5000, None, 0x6000, None, None, None) == _capi.ERR_ARG
    store = lib.cslbm_step_store
    assert store(C.byref(L), -1, None, None, None) == _capi.ERR_ARG
    assert store(C.byref(L), 2, None, None, None) == _capi.ERR_ARG
    states = (C.c_void_p * 2)(0x1000, 0x7000)       # the first aliases L->f
    assert store(C.byref(L), 2, states, None, None) == _capi.ERR_ARG
    assert store(C.byref(L), 0, None, None, None) == _capi.OK


def test_gradient_mode_argument_checks(lib):
    assert lib.cslbm_step(C.byref(make_level(p_grad_mode=2)), 1, None) == _capi.ERR_ARG
    assert "grad_mode" in err(lib)
    assert lib.cslbm_step(C.byref(make_level(p_grad_mode=1)), 1, None) == _capi.ERR_ARG
    assert "vel" in err(lib)
    flagged = make_level(p_grad_mode=1, flags=0x9000, vel=0xB000, vel_next=0xC000)
    assert lib.cslbm_step(C.byref(flagged), 1, None) == _capi.ERR_UNSUPPORTED


def test_multiscale_adjoint_argument_checks(lib):
    ab, adj = lib.cslbm_multiscale_adjoint_bytes, lib.cslbm_multiscale_adjoint_step
    L0 = make_level(dx=1.0)
    L1 = make_level(dx=0.5, flags=0x9000, periodic=0)
    L2 = make_level(dx=0.25, flags=0x9100, periodic=0)
    H, keep = hierarchy_of([L0, L1, L2], [-1, 0, 1])
    n = ab(C.byref(H))
    assert n > 0
    ptrs = (C.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    assert adj(C.byref(H), ptrs, None, ptrs, None, None, n, None) == _capi.ERR_ARG
    assert "workspace" in err(lib)
    assert adj(C.byref(H), ptrs, None, ptrs, None, 0xF000, n - 1, None) == _capi.ERR_ARG
    assert adj(C.byref(H), None, None, ptrs, None, 0xF000, n, None) == _capi.ERR_ARG
    # not a chain
    H, keep = hierarchy_of([L0, L1, L2], [-1, 0, 0])
    assert ab(C.byref(H)) == -1
    assert "chain" in err(lib)
    assert adj(C.byref(H), ptrs, None, ptrs, None, 0xF000, n, None) == _capi.ERR_UNSUPPORTED
    # binary16 storage
    H, keep = hierarchy_of([L0, make_level(dx=0.5, flags=0x9000, periodic=0, storage=_capi.F16S)],
                           [-1, 0])
    assert ab(C.byref(H)) == -1
    assert "FP32" in err(lib)
    # a far-field scale
    H, keep = hierarchy_of([L0, make_level(dx=2.0, flags=0x9000, periodic=0)], [-1, 0])
    assert ab(C.byref(H)) == -1


def test_wall_cell_count_checked_and_adjoints_refuse_wall_nodes(lib):
    """wall_cells must be >= 0 and needs a flags array; the adjoint calls do
    not differentiate wall nodes and refuse a level that has them (all
    before any launch)."""
    L = make_level(wall_cells=-1)
    assert lib.cslbm_step(C.byref(L), 1, None) == _capi.ERR_ARG
    L = make_level(wall_cells=4)
    assert lib.cslbm_step(C.byref(L), 1, None) == _capi.ERR_ARG
    assert "wall_cells" in err(lib)
    L = make_level(wall_cells=4, flags=0x9000, periodic=3)
    assert lib.cslbm_adjoint_step(C.byref(L), 0x5000, None, 0x6000, None, None, None) == \
        _capi.ERR_UNSUPPORTED
    assert "wall" in err(lib)
