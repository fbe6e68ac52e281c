"""GPU parity of sparse brick storage (8x8x8 bricks, only the bricks of a
region stored) against the FP64 oracle run on the whole box, where the
cells outside the stored bricks are SOLID: a single brick level over
several steps (fluid, ghost layer, a solid sphere, scalar with buoyancy),
and hierarchies in which a finer scale is brick-stored, as the target of
prior-mapping and post-mapping and as the parent of a dense finer scale."""
import numpy as np
import pytest
import torch

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import _capi, hierarchy, inputs
from paper_1807_02284_amd.level import F16S, F32, Level, Params
from test_parity_multiscale import Spec, smooth_state

pytestmark = pytest.mark.gpu

W = oracle.weights()


def rel_err(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), W[:, None]))


def ball(shape, centre, radius, origin=(0.0, 0.0, 0.0), dx=1.0):
    nx, ny, nz = shape
    px = origin[0] + np.arange(nx) * dx
    py = origin[1] + np.arange(ny) * dx
    pz = origin[2] + np.arange(nz) * dx
    return ((px[None, None, :] - centre[0]) ** 2 + (py[None, :, None] - centre[1]) ** 2 +
            (pz[:, None, None] - centre[2]) ** 2) <= radius ** 2


def storage_pop(lev: Level):
    h = lev.f.reshape(27, lev.plane)[:, : lev.n].double().cpu().numpy()
    return h + W[:, None]


def storage_g(lev: Level):
    return lev.g.reshape(7, lev.plane)[:, : lev.n].double().cpu().numpy()


@pytest.mark.parametrize("storage", [F32, F16S])
def test_brick_level_steps_match_oracle(storage):
    shape = (40, 32, 24)
    region = ball(shape, (20.0, 15.0, 11.0), 11.0)
    solid = ball(shape, (21.0, 16.0, 12.0), 3.0)
    bricks, kinds = hierarchy.brick_kinds(region, solid)
    assert 0 < bricks.sum() < bricks.size
    p = Params(nu=5e-3, g_max=0.1, tau_s=0.6, beta=1e-3, s_ref=0.5)
    lev = Level(*shape, p, scalar=True, flags=kinds, bricks=bricks, storage=storage)
    n = int(np.prod(shape))
    x, y, z = inputs.grid_coords(*shape)
    rho = 1.0 + 0.01 * np.sin(2 * np.pi * (x + 2 * y) / 24.0)
    u = np.stack([0.03 * np.cos(2 * np.pi * (y + z) / 16.0), 0.02 * np.sin(2 * np.pi * x / 20.0),
                  0.01 * np.cos(2 * np.pi * (x - y) / 12.0)]) + 0.002 * inputs.perturbation((3, n), 5)
    s = 0.5 + 0.2 * np.cos(2 * np.pi * (x - z) / 14.0)
    lev.init_equilibrium(lev.to_storage(rho), lev.to_storage(u), lev.to_storage(s))
    dom = oracle.Domain(*shape, periodic=0, flags=kinds)
    f, g = oracle.init(dom, rho, u, s=s)
    # both sides start from the stored FP32/FP16 values
    f[:, lev.dense_index] = storage_pop(lev)
    g[:, lev.dense_index] = storage_g(lev)
    steps = 5 if storage == F32 else 1
    lev.step(steps)
    torch.cuda.synchronize()
    op = oracle.Params(nu=p.nu, g_max=p.g_max, tau_s=p.tau_s, beta=p.beta, s_ref=p.s_ref)
    ref, gref = oracle.step(dom, op, f, g, n_steps=steps)
    got, gg = storage_pop(lev), storage_g(lev)
    if storage == F32:
        assert rel_err(got, ref[:, lev.dense_index]) <= 5e-6
        assert np.max(np.abs(gg - gref[:, lev.dense_index])) <= 5e-6
    else:
        # binary16 storage of f - w: a few half-precision ulps of the largest |f - w|
        h = ref[:, lev.dense_index] - W[:, None]
        bound = 4 * 2.0 ** -11 * np.max(np.abs(h)) + 1e-7
        assert np.max(np.abs(got - ref[:, lev.dense_index])) <= bound
    # the cells outside the stored bricks are never read: the layer of GHOST
    # cells keeps every FLUID cell's neighbours stored
    k3 = kinds.reshape(shape[2], shape[1], shape[0])
    stored = bricks.repeat(8, 0).repeat(8, 1).repeat(8, 2)
    assert np.all(stored[k3 == _capi.FLUID])


def _spec_with(shape, origin, dx, nu0, kinds, parent):
    return Spec(shape, origin, dx, nu0, kinds, parent=parent)


@pytest.mark.parametrize("n_scales,brick2", [(2, False), (3, False), (3, True)])
def test_hierarchy_with_a_brick_scale_matches_oracle(n_scales, brick2):
    """Reference 32^3 periodic (dense); scale 1 brick-stored over a ball at
    spacing 2/3; with three scales, scale 2 at spacing 1/2 inside scale 1's
    fluid (its parent and post-mapping target is the brick scale), as a
    dense box or itself brick-stored over a smaller ball (exchanges between
    two brick levels)."""
    n = 32
    nu0 = 2e-3
    s0 = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    centre = (16.2, 15.7, 16.4)
    lo1, hi1, r1 = ((4.0,) * 3, (28.0,) * 3, 10.0) if brick2 else ((5.0,) * 3, (27.0,) * 3, 8.5)
    lev1, kinds1 = hierarchy.brick_scale(lo1, hi1, 1.5, s0.params(),
                                         lambda px, py, pz: (px - centre[0]) ** 2 + (py - centre[1]) ** 2
                                         + (pz - centre[2]) ** 2 <= r1 ** 2,
                                         scalar=True, storage=F32)
    assert lev1.n_bricks < (lev1.nx // 8) * (lev1.ny // 8) * (lev1.nz // 8)
    s1 = _spec_with((lev1.nx, lev1.ny, lev1.nz), tuple(lev1.c.origin), lev1.c.dx, nu0, kinds1, 0)
    specs = [s0, s1]
    levs = [s0.level(True), lev1]
    if n_scales == 3 and not brick2:
        sh2 = (14, 13, 12)
        s2 = Spec(sh2, (13.1, 12.8, 13.3), 0.5, nu0, hierarchy.shell_flags(*sh2), parent=1)
        specs.append(s2)
        levs.append(s2.level(True))
    elif n_scales == 3:
        lev2, kinds2 = hierarchy.brick_scale((11.0, 11.0, 11.0), (21.0, 21.0, 21.0), 2.0, s0.params(),
                                             lambda px, py, pz: (px - centre[0]) ** 2 + (py - centre[1]) ** 2
                                             + (pz - centre[2]) ** 2 <= 3.0 ** 2,
                                             scalar=True, storage=F32)
        assert lev2.n_bricks < (lev2.nx // 8) * (lev2.ny // 8) * (lev2.nz // 8)
        specs.append(_spec_with((lev2.nx, lev2.ny, lev2.nz), tuple(lev2.c.origin), lev2.c.dx, nu0,
                                kinds2, 1))
        levs.append(lev2)
    oscs = []
    for sp, lev in zip(specs, levs):
        rho, u, s = smooth_state(sp, 50)
        lev.init_equilibrium(lev.to_storage(rho), lev.to_storage(u), lev.to_storage(s))
        osc = sp.oscale()
        osc.f, osc.g = oracle.init(osc.domain(), rho, u, s=s)
        idx = lev.dense_index if lev.dense_index is not None else np.arange(lev.n)
        osc.f[:, idx] = storage_pop(lev)
        osc.g[:, idx] = storage_g(lev)
        oscs.append(osc)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs])
    ml.prepare(oscs)
    for (i, j), cells in H.post_full.items():
        np.testing.assert_array_equal(np.sort(cells.astype(np.int64)), oscs[i].post[j])
    H.step(3)
    ml.multiscale_step(oscs, 3)
    torch.cuda.synchronize()
    for lev, osc in zip(levs, oscs):
        idx = lev.dense_index if lev.dense_index is not None else np.arange(lev.n)
        assert rel_err(storage_pop(lev), osc.f[:, idx]) <= 1e-5
        assert np.max(np.abs(storage_g(lev) - osc.g[:, idx])) <= 1e-5


def test_brick_level_rejections():
    shape = (16, 16, 16)
    bricks, kinds = hierarchy.brick_kinds(ball(shape, (8.0, 8.0, 8.0), 5.0))
    lev = Level(*shape, Params(nu=1e-2), flags=kinds, bricks=bricks)
    with pytest.raises(_capi.CslbmError):
        lev.vorticity()
    lam = torch.zeros(27 * lev.plane, device="cuda")
    with pytest.raises(_capi.CslbmError):
        lev.adjoint_step(lev.f, None, lam, None, torch.zeros_like(lam), None, None)
