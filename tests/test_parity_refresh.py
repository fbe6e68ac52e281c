"""Rebuilding dynamic regions (section "Scale construction": dynamic scales
are rebuilt every 40 iterations): kept cells carry their state over bit for
bit, new cells take the parent's mapped state, and the rebuilt hierarchy
steps in parity with the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import hierarchy, inputs
from paper_1807_02284_amd.level import Level, Params
from test_parity_multiscale import gpu_g, gpu_pop, rel_err

pytestmark = pytest.mark.gpu


def test_rebuilt_regions_keep_shared_cells_and_step_in_parity():
    nx, ny, nz = 96, 48, 48
    sc = nx / 512.0
    kinds0 = inputs.plume_flags(nx, ny, nz)
    centre, r = (160.0 * sc, ny / 2.0, nz / 2.0), 24.0 * sc

    def sphere(px, py, pz):
        return (px + 0.5 - centre[0]) ** 2 + (py + 0.5 - centre[1]) ** 2 + (pz + 0.5 - centre[2]) ** 2 <= r * r

    p0 = Params(nu=1e-3, g_max=0.05, tau_s=0.55, u_in=(0.06, 0.0, 0.0), s_in=1.0)
    lev0 = Level(nx, ny, nz, p0, scalar=True, periodic=0, flags=kinds0)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    jet = ((y + 0.5 - ny / 2) ** 2 + (z + 0.5 - nz / 2) ** 2 <= (32 * sc) ** 2) & (kinds0 == 0)
    u = np.zeros((3, x.size))
    u[0, jet] = 0.06
    lev0.init_equilibrium(None, u, np.where(jet, 1.0, 0.0))
    lev0.step(60)
    thr = ((1e-3, 0.005), (4e-3, 0.01))
    H1, boxes1 = hierarchy.dynamic_hierarchy(lev0, kinds0, thr, (1.5, 2.0), solid_fn=sphere, margin=4)
    assert len(H1.levels) == 3
    H1.step(10)
    torch.cuda.synchronize()
    old = [gpu_pop(lv) for lv in H1.levels[1:]]
    # rebuild with tighter thresholds, so that the regions surely move
    thr2 = ((2e-3, 0.01), (8e-3, 0.02))
    H2, boxes2 = hierarchy.dynamic_hierarchy(lev0, kinds0, thr2, (1.5, 2.0), solid_fn=sphere,
                                             margin=4, previous=H1)
    assert len(H2.levels) == 3 and boxes2 != boxes1
    for i in (1, 2):
        src, dst = hierarchy.kept_cells(H1.levels[i], H1.kinds[i], H2.levels[i], H2.kinds[i])
        assert src.size > 0
        np.testing.assert_array_equal(gpu_pop(H2.levels[i])[:, dst], old[i - 1][:, src])
    # the rebuilt hierarchy against the oracle from the same state
    oscs = []
    for i, (lev, k) in enumerate(zip(H2.levels, H2.kinds)):
        p = lev.params
        osc = ml.OScale(lev.nx, lev.ny, lev.nz, lev.c.dx, tuple(lev.c.origin),
                        oracle.Params(nu=p.nu, g_max=p.g_max, tau_s=p.tau_s), k, periodic=0,
                        parent=H2.parents[i], u_in=p.u_in, s_in=p.s_in)
        osc.f, osc.g = gpu_pop(lev), gpu_g(lev)
        oscs.append(osc)
    ml.prepare(oscs)
    H2.step(4)
    ml.multiscale_step(oscs, 4)
    torch.cuda.synchronize()
    for lev, osc in zip(H2.levels, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5
