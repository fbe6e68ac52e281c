"""A hierarchy built by the static scale construction (distance map and
inlet shadow) runs Algorithm 1 on the GPU in parity with the FP64 oracle
given the same scales, cell kinds and initial states."""
import numpy as np
import pytest
import torch

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import hierarchy, inputs
from paper_1807_02284_amd.level import Level, Params
from test_parity_multiscale import gpu_g, gpu_pop, rel_err

pytestmark = pytest.mark.gpu


def test_static_hierarchy_of_the_reduced_plume_matches_oracle():
    nx, ny, nz = 96, 48, 48
    sc = nx / 512.0
    kinds0 = inputs.plume_flags(nx, ny, nz)
    centre, r = (160.0 * sc, ny / 2.0, nz / 2.0), 24.0 * sc

    def sphere(px, py, pz):
        return (px + 0.5 - centre[0]) ** 2 + (py + 0.5 - centre[1]) ** 2 + (pz + 0.5 - centre[2]) ** 2 <= r * r

    p0 = Params(nu=1e-3, g_max=0.05, tau_s=0.55, u_in=(0.05, 0.0, 0.0), s_in=1.0)
    lev0 = Level(nx, ny, nz, p0, scalar=True, periodic=0, flags=kinds0)
    x, y, _ = inputs.grid_coords(nx, ny, nz)
    u = np.zeros((3, x.size))
    u[0] = 0.03 * (kinds0 == 0)
    s = 0.5 + 0.3 * np.cos(2 * np.pi * (x + y) / 24.0)
    lev0.init_equilibrium(None, u, s)
    H, boxes, spacings = hierarchy.static_hierarchy(
        lev0, kinds0, 3, 0.5, 6.0, faces=False, inlet_center=(ny / 2.0, nz / 2.0),
        inlet_radius=32.0 * sc, solid_fn=sphere, margin=4)
    assert len(H.levels) == 3 and spacings == [0.75, 0.5]
    oscs = []
    for i, (lev, k) in enumerate(zip(H.levels, H.kinds)):
        p = lev.params
        osc = ml.OScale(lev.nx, lev.ny, lev.nz, lev.c.dx, tuple(lev.c.origin),
                        oracle.Params(nu=p.nu, g_max=p.g_max, tau_s=p.tau_s), k, periodic=0,
                        parent=H.parents[i], u_in=p.u_in, s_in=p.s_in)
        osc.f, osc.g = gpu_pop(lev), gpu_g(lev)
        oscs.append(osc)
    ml.prepare(oscs)
    for (i, j), cells in H.post_full.items():
        np.testing.assert_array_equal(np.sort(cells.astype(np.int64)), oscs[i].post[j])
    H.step(6)
    ml.multiscale_step(oscs, 6)
    torch.cuda.synchronize()
    for lev, osc in zip(H.levels, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5
