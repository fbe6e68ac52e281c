"""GPU parity of far-field scales (spacing larger than the reference scale)
and of the Neumann far-field boundary against the FP64 oracle, on the same
seeded fields and the same scale geometry (masks given to both sides)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import _capi, hierarchy, inputs
from test_parity_multiscale import Spec, gpu_g, gpu_pop, rel_err, start_both

pytestmark = pytest.mark.gpu


def window_kinds(shape):
    return hierarchy.shell_flags(*shape)


def far_kinds(shape, origin, dx, window: Spec):
    """GHOST where the trilinear stencil in the window is made of its FLUID
    cells (oracle's own rule), NEUMANN on the faces, FLUID elsewhere."""
    n = int(np.prod(shape))
    probe = ml.OScale(*shape, dx, origin, oracle.Params(), np.zeros(n, np.uint8))
    win = ml.OScale(*window.shape, window.dx, window.origin, oracle.Params(), window.kinds)
    kinds = np.zeros(n, np.uint8)
    kinds[ml.post_targets(probe, win)] = oracle.GHOST
    x, y, z = inputs.grid_coords(*shape)
    face = (x == 0) | (x == shape[0] - 1) | (y == 0) | (y == shape[1] - 1) | (z == 0) | (z == shape[2] - 1)
    kinds[face] = oracle.NEUMANN
    return kinds


def build(specs, seed):
    levs, oscs = [], []
    for sp in specs:
        lev, osc = start_both(sp, seed)
        levs.append(lev)
        oscs.append(osc)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs])
    ml.prepare(oscs)
    for i, sp in enumerate(specs[1:], start=1):
        np.testing.assert_array_equal(H.ghost_cells(i), oscs[i].ghosts)
        for j, cells in oscs[i].post.items():
            np.testing.assert_array_equal(np.sort(H.post_full[(i, j)].astype(np.int64)), cells)
    return H, levs, oscs


def test_neumann_faces_single_level_match_oracle():
    shape = (13, 11, 9)
    kinds = np.zeros(int(np.prod(shape)), np.uint8)
    x, y, z = inputs.grid_coords(*shape)
    kinds[(x == 0) | (x == 12) | (y == 0) | (y == 10) | (z == 0) | (z == 8)] = oracle.NEUMANN
    sp = Spec(shape, (0.0, 0.0, 0.0), 1.0, 2e-3, kinds)
    lev, osc = start_both(sp, 31)
    lev.step(3)
    f, g = oracle.step(osc.domain(), osc.params, osc.f, osc.g, n_steps=3)
    torch.cuda.synchronize()
    assert rel_err(gpu_pop(lev), f) <= 1e-6
    assert np.max(np.abs(gpu_g(lev) - g)) <= 1e-6


@pytest.mark.parametrize("dxc,shape_c", [(2.0, (21, 19, 17)), (4.0 / 3.0, (31, 28, 25))])
def test_far_field_and_reference_window_match_oracle(dxc, shape_c):
    nu0 = 2e-3
    wshape = (20, 18, 16)
    win = Spec(wshape, (10.0, 9.0, 8.0), 1.0, nu0, window_kinds(wshape))
    far = Spec(shape_c, (0.0, 0.0, 0.0), dxc, nu0, far_kinds(shape_c, (0.0, 0.0, 0.0), dxc, win),
               parent=0)
    H, levs, oscs = build([win, far], 41)
    assert H.far == [False, True]
    H.step(4)
    ml.multiscale_step(oscs, 4)
    torch.cuda.synchronize()
    for lev, osc in zip(levs, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5


def test_far_field_reference_and_finer_scale_match_oracle():
    """Three scales: a far field (spacing 2) around the reference window,
    and a finer scale (spacing 1/2) inside the window."""
    nu0 = 2e-3
    wshape = (22, 20, 18)
    win = Spec(wshape, (10.0, 9.0, 8.0), 1.0, nu0, window_kinds(wshape))
    fshape = (14, 13, 12)
    fine = Spec(fshape, (16.0, 15.0, 14.0), 0.5, nu0, hierarchy.shell_flags(*fshape), parent=0)
    shape_c = (22, 20, 18)
    far = Spec(shape_c, (0.0, 0.0, 0.0), 2.0, nu0, far_kinds(shape_c, (0.0, 0.0, 0.0), 2.0, win),
               parent=0)
    H, levs, oscs = build([win, fine, far], 42)
    H.step(3)
    ml.multiscale_step(oscs, 3)
    torch.cuda.synchronize()
    for lev, osc in zip(levs, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5


def test_far_field_post_map_rejected_onto_other_scales():
    """The driver refuses a far-field scale that post-maps anywhere but its
    parent's shell (argument check before any launch)."""
    nu0 = 2e-3
    wshape = (12, 12, 12)
    win = Spec(wshape, (6.0, 6.0, 6.0), 1.0, nu0, window_kinds(wshape))
    shape_c = (13, 13, 13)
    far = Spec(shape_c, (0.0, 0.0, 0.0), 2.0, nu0, far_kinds(shape_c, (0.0, 0.0, 0.0), 2.0, win),
               parent=0)
    H, levs, oscs = build([win, far], 43)
    H.c_scales[1].n_post[1] = 5
    H.c_scales[1].post_cells[1] = H.c_scales[1].post_cells[0]
    with pytest.raises(_capi.CslbmError):
        H.step(1)
