"""GPU parity of the no-slip wall node (kind WALL: the regularized wall
through the node, Latt & Chopard 2006; Latt et al., Phys. Rev. E 77, 056703,
2008) against the FP64 oracle on the same seeded inputs, and its rejection
rules."""
import numpy as np
import pytest
import torch

import oracle
from paper_1807_02284_amd import _capi, inputs
from paper_1807_02284_amd.level import Level, Params
from test_parity_single import gpu_f64, odomain, oparams, perturbed_start, rel_err, start_fields

pytestmark = pytest.mark.gpu


def wall_kinds(nx, ny, nz, sphere=False):
    """Walls through the nodes z = 0 and z = nz - 1 (periodic in x and y);
    optionally a solid ball in the middle (its neighbours bounce back)."""
    kinds = np.zeros(nx * ny * nz, np.uint8)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    kinds[(z == 0) | (z == nz - 1)] = _capi.WALL
    if sphere:
        r2 = (x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2
        kinds[r2 <= 2.2 ** 2] = _capi.SOLID
    return kinds


@pytest.mark.parametrize("nx,ny,nz,seed", [(70, 9, 7, 1), (33, 17, 6, 2)])
def test_one_step_with_wall_nodes_and_force_matches_oracle(nx, ny, nz, seed):
    n = nx * ny * nz
    p = Params(nu=0.01, g_max=0.05)
    kinds = wall_kinds(nx, ny, nz)
    force = inputs.smooth_random_field(nx, ny, nz, 2e-4, seed + 20)
    rho, u = start_fields(nx, ny, nz, seed, u_amp=0.05)
    noise = 2e-4 * inputs.perturbation((27, n), seed + 4)
    lev = Level(nx, ny, nz, p, periodic=3, flags=kinds, force=force)
    assert lev.wall_cells == 2 * nx * ny
    dom = odomain(nx, ny, nz, periodic=3, flags=kinds, theta=force)
    f0, _ = perturbed_start(lev, dom, rho, u, noise)
    lev.step(1)
    f1, _ = oracle.step(dom, oparams(p), f0)
    got, _ = gpu_f64(lev)
    assert rel_err(got, f1) <= 1e-6


def test_ten_steps_with_walls_solid_ball_scalar_and_buoyancy_match_oracle():
    nx, ny, nz = 40, 12, 11
    n = nx * ny * nz
    s0 = 0.5 + 0.4 * inputs.smooth_random_field(nx, ny, nz, 1.0, 31)[0]
    p = Params(nu=0.005, g_max=0.05, tau_s=0.6, beta=1e-3, s_ref=float(s0.mean()))
    kinds = wall_kinds(nx, ny, nz, sphere=True)
    rho, u = start_fields(nx, ny, nz, 5, u_amp=0.04)
    u[:, kinds == _capi.SOLID] = 0.0
    noise = 1e-4 * inputs.perturbation((27, n), 9)
    lev = Level(nx, ny, nz, p, periodic=3, flags=kinds, scalar=True)
    dom = odomain(nx, ny, nz, periodic=3, flags=kinds, p=p)
    f0, g0 = perturbed_start(lev, dom, rho, u, noise, s=s0)
    lev.step(10)
    f10, g10 = oracle.step(dom, oparams(p), f0, g0, n_steps=10)
    got, gg = gpu_f64(lev)
    fluid = kinds != _capi.SOLID
    assert rel_err(got[:, fluid], f10[:, fluid]) <= 1e-5
    assert np.max(np.abs(gg[:, fluid] - g10[:, fluid])) <= 1e-5


def test_force_driven_channel_reaches_the_oracle_steady_state():
    """Walls through the nodes y = 0 and y = N - 1, uniform force along x:
    after 6000 steps the GPU profile equals the oracle's steady state, which
    is pinned on the CPU to the closed-form parabola at second order."""
    N, nu, F, steps = 17, 0.3, 1e-6, 6000
    kinds = np.zeros(N, np.uint8)
    kinds[0] = kinds[-1] = _capi.WALL
    th = np.zeros((3, N))
    th[0] = F
    p = Params(nu=nu, g_max=0.1)
    lev = Level(1, N, 1, p, periodic=5, flags=kinds, force=th)
    lev.init_equilibrium(np.ones(N), np.zeros((3, N)))
    lev.step(steps)
    _, ug, _ = lev.read_macro()
    ug = ug.double().cpu().numpy()
    dom = odomain(1, N, 1, periodic=5, flags=kinds, theta=th)
    f, _ = oracle.init(dom, np.ones(N), np.zeros((3, N)))
    f, _ = oracle.step(dom, oparams(p), f, n_steps=steps)
    _, uo, _ = oracle.macro(dom, oparams(p), f)
    assert np.max(np.abs(ug[0] - uo[0])) <= 1e-5 * np.max(uo[0])
    assert abs(ug[0, 0]) <= 1e-6 * np.max(uo[0]) and abs(ug[0, -1]) <= 1e-6 * np.max(uo[0])


def test_wall_node_off_a_flat_wall_is_flagged_nonfinite_and_adjoint_rejects_walls():
    """A WALL node in a corner (blocked along y and z) is not on one flat
    wall: its normal code is 7 and the step writes NaN there, which the
    finiteness check reports.  The adjoint refuses levels with wall nodes."""
    nx, ny, nz = 4, 6, 6
    kinds = np.zeros(nx * ny * nz, np.uint8)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    kinds[(y == 0) | (z == 0)] = _capi.WALL
    lev = Level(nx, ny, nz, Params(nu=0.1), periodic=1, flags=kinds)
    fl = lev.flags[: lev.n].cpu().numpy()
    codes = fl >> _capi.WALL_NORMAL_SHIFT
    corner = (y == 0) & (z == 0)
    assert np.all(codes[corner] == 7)
    assert np.all(codes[(y == 0) & (z > 0) & (z < nz - 1)] == 3)
    assert np.all(codes[(z == 0) & (y > 0) & (y < ny - 1)] == 5)
    assert np.all(codes[kinds != _capi.WALL] == 0)
    lev.init_equilibrium(np.ones(lev.n), np.zeros((3, lev.n)))
    lev.step(1)
    assert lev.count_nonfinite() > 0
    with pytest.raises(_capi.CslbmError):
        z0 = torch.zeros(27 * lev.plane, device="cuda")
        lev.adjoint_step(lev.f, None, z0, None, torch.zeros_like(z0), None, None)


def test_wall_nodes_with_binary16_storage_within_rounding_bound():
    """Binary16 storage of f - w with wall nodes: one step against the oracle
    started from the same stored values, within the rounding of the output
    to binary16 (half an ulp of |h|, or the subnormal spacing) plus FP32."""
    from paper_1807_02284_amd.level import F16S
    nx, ny, nz = 40, 9, 8
    n = nx * ny * nz
    p = Params(nu=0.01, g_max=0.05)
    kinds = wall_kinds(nx, ny, nz)
    force = inputs.smooth_random_field(nx, ny, nz, 2e-4, 44)
    rho, u = start_fields(nx, ny, nz, 8, u_amp=0.05)
    dom = odomain(nx, ny, nz, periodic=3, flags=kinds, theta=force)
    feq, _ = oracle.init(dom, rho, u)
    W = oracle.weights()
    h16 = (feq - W[:, None] + 2e-4 * inputs.perturbation((27, n), 45)).astype(np.float16)
    lev = Level(nx, ny, nz, p, storage=F16S, periodic=3, flags=kinds, force=force)
    lev.set_populations(torch.as_tensor(h16.astype(np.float32)), shifted=True)
    lev.step(1)
    f1, _ = oracle.step(dom, oparams(p), h16.astype(np.float64) + W[:, None])
    got, _ = gpu_f64(lev)
    bound = np.abs(f1 - W[:, None]) * 2.0 ** -11 + 2.0 ** -25 + 2e-7 * np.abs(f1)
    assert np.all(np.abs(got - f1) <= bound)
