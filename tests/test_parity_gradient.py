"""GPU parity of the finite-difference gradient mode of the adaptive
relaxation (grad_mode 1: |grad u|_F of the stored velocity field, one step
lagged) against the FP64 oracle, small sizes and the 256^3 benchmark field."""
import numpy as np
import pytest
import torch

import oracle
from paper_1807_02284_amd import _capi, inputs
from paper_1807_02284_amd.level import F32, Level, Params
from test_parity_single import gpu_f64, oparams, rel_err, start_fields

pytestmark = pytest.mark.gpu

W = oracle.weights()


def oparams_grad(p: Params) -> oracle.Params:
    op = oparams(p)
    op.grad_mode = p.grad_mode
    return op


@pytest.mark.parametrize("g_max", [0.022, 0.1])
def test_gradient_mode_ten_steps_match_oracle(g_max):
    """Smooth seeded start with per-cell noise (|grad u| from 0.004 to 0.042,
    median 0.022): g_max 0.022 puts about half of the box on the clamp, 0.1
    none of it."""
    nx, ny, nz = 40, 18, 11
    n = nx * ny * nz
    p = Params(nu=2e-3, g_max=g_max, grad_mode=1)
    rho, u = start_fields(nx, ny, nz, 61, u_amp=0.05)
    noise = 1e-4 * W[:, None] * inputs.perturbation((27, n), 62)
    dom = oracle.Domain(nx, ny, nz)
    f0, _ = oracle.init(dom, rho, u)
    f0 = f0 + noise
    lev = Level(nx, ny, nz, p)
    lev.set_populations(f0 - W[:, None], shifted=True)
    G = oracle.grad_field(dom, oparams_grad(p), f0)
    if g_max < 0.05:
        assert np.mean(G > g_max) > 0.3 and np.mean(G < g_max) > 0.3
    else:
        assert np.all(G < g_max)
    lev.step(10)
    ref, _ = oracle.step(dom, oparams_grad(p), f0, n_steps=10)
    got, _ = gpu_f64(lev)
    assert rel_err(got, ref) <= 5e-6
    # the stored velocity field is the read-back velocity of the state
    _, uref, _ = oracle.macro(dom, oparams_grad(p), ref)
    vel = lev.vel.reshape(3, n).double().cpu().numpy()
    assert np.max(np.abs(vel - uref)) <= 1e-6


def test_gradient_mode_with_force_and_scalar_matches_oracle():
    nx, ny, nz = 24, 20, 12
    n = nx * ny * nz
    s0 = 0.5 + 0.3 * inputs.smooth_random_field(nx, ny, nz, 1.0, 71, k_max=2)[0]
    theta = inputs.smooth_random_field(nx, ny, nz, 2e-4, 72, k_max=2)
    p = Params(nu=5e-3, g_max=0.01, tau_s=0.6, beta=1e-3, s_ref=float(s0.mean()), grad_mode=1)
    rho, u = start_fields(nx, ny, nz, 73, u_amp=0.04)
    dom = oracle.Domain(nx, ny, nz, theta=theta)
    f0, g0 = oracle.init(dom, rho, u, s=s0)
    lev = Level(nx, ny, nz, p, scalar=True, force=theta)
    lev.set_populations(f0 - W[:, None], g0, shifted=True)
    lev.step(5)
    ref, gref = oracle.step(dom, oparams_grad(p), f0, g0, n_steps=5)
    got, gg = gpu_f64(lev)
    assert rel_err(got, ref) <= 5e-6
    assert np.max(np.abs(gg - gref)) <= 1e-6


def test_gradient_mode_full_size_256_first_step_sampled():
    """The 256^3 benchmark field in gradient mode, one step, 400 sampled
    cells against the oracle (which takes the gradient of the whole
    field)."""
    n = 256
    N = n ** 3
    p = Params(nu=1e-5, g_max=0.1, grad_mode=1)
    rho, u = inputs.turbulence(n, 2, 32, 0.04, seed=1807)
    lev = Level(n, n, n, p)
    lev.init_equilibrium(rho, u)
    h0, _ = lev.get_populations(shifted=True)
    f0 = h0.double().cpu().numpy() + W[:, None]        # the exact FP32 start, both sides
    del h0
    lev.step(1)
    rng = np.random.default_rng(256)
    cells = np.unique(rng.integers(0, N, 400))
    dom = oracle.Domain(n, n, n)
    ref, _ = oracle.step_cells(dom, oparams_grad(p), f0, cells)
    h, _ = lev.get_populations(shifted=True)
    got = h[:, torch.as_tensor(cells, device=h.device)].double().cpu().numpy() + W[:, None]
    del lev, h
    torch.cuda.empty_cache()
    assert rel_err(got, ref) <= 1e-6


def test_gradient_mode_rejects_flagged_levels_and_other_paths():
    n = 8
    flags = np.zeros(n ** 3, np.uint8)
    lev = Level(n, n, n, Params(nu=1e-3, grad_mode=1), flags=flags)
    lev.init_equilibrium(None, np.zeros((3, n ** 3)))
    with pytest.raises(_capi.CslbmError):
        lev.step(1)
    lev2 = Level(n, n, n, Params(nu=1e-3, grad_mode=1))
    lev2.init_equilibrium(None, np.zeros((3, n ** 3)))
    lam = torch.zeros(27 * lev2.plane, device="cuda")
    with pytest.raises(_capi.CslbmError):
        lev2.adjoint_step(lev2.f, None, lam, None, torch.zeros_like(lam), None, None)


def test_gradient_mode_running_maximum_matches_oracle():
    """g_max of every step = the maximum of that step's gradient field
    (reduced on the GPU before the step)."""
    nx, ny, nz = 40, 18, 11
    n = nx * ny * nz
    p = Params(nu=2e-3, g_max=0.05, grad_mode=1, gmax_running=True)
    rho, u = start_fields(nx, ny, nz, 81, u_amp=0.05)
    dom = oracle.Domain(nx, ny, nz)
    f0, _ = oracle.init(dom, rho, u)
    lev = Level(nx, ny, nz, p)
    lev.set_populations(f0 - W[:, None], shifted=True)
    lev.step(10)
    op = oparams_grad(p)
    op.gmax_running = True
    f9, _ = oracle.step(dom, op, f0, n_steps=9)
    gmax9 = float(oracle.grad_field(dom, op, f9).max())
    ref, _ = oracle.step(dom, op, f9, n_steps=1)
    got, _ = gpu_f64(lev)
    assert rel_err(got, ref) <= 5e-6
    assert float(lev.gmax_buf[-1]) == pytest.approx(gmax9, rel=1e-5)
