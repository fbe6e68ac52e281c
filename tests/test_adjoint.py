"""GPU adjoint (hand-written VJP of the collide-stream step behind a
torch.autograd.Function with checkpoint-every-K recomputation) against
central finite differences of the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1807_02284_amd import inputs
from paper_1807_02284_amd.level import Level, Params
from paper_1807_02284_amd.rollout import rollout

pytestmark = pytest.mark.gpu

N1 = 16
W = oracle.weights()
TARGET_STEPS = 12


def scene(adaptive=True, g_max=1.0):
    n = N1
    s0 = inputs.gaussian_blob(n, n, n, (8, 8, 4), 1.5)
    p = Params(nu=0.01, g_max=g_max, adaptive=adaptive, tau_s=0.55, beta=1e-3,
               s_ref=float(s0.mean()))
    u0 = inputs.smooth_random_field(n, n, n, 0.02, 51, k_max=2)
    theta = inputs.smooth_random_field(n, n, n, 1e-4, 52, k_max=2)
    # the target: final smoke scalar of a seeded target run, the same scene
    # driven by another smooth body force for TARGET_STEPS steps (FP64
    # oracle; strong enough that s - target stays far above FP32 rounding)
    theta_t = inputs.smooth_random_field(n, n, n, 1e-3, 53, k_max=2)
    dom = oracle.Domain(n, n, n, theta=theta_t)
    op = oracle.Params(nu=p.nu, g_max=p.g_max, adaptive=p.adaptive, tau_s=p.tau_s, beta=p.beta,
                       s_ref=p.s_ref)
    f, g = oracle.init(dom, np.ones(n ** 3), u0, s=s0)
    f, g = oracle.step(dom, op, f, g, n_steps=TARGET_STEPS)
    _, _, target = oracle.macro(dom, op, f, g)
    return p, u0, s0, theta, target


def oracle_loss(p, u0, s0, theta, target, n_steps, dh=None, dg=None):
    n = N1
    dom = oracle.Domain(n, n, n, theta=theta)
    op = oracle.Params(nu=p.nu, g_max=p.g_max, adaptive=p.adaptive, tau_s=p.tau_s, beta=p.beta,
                       s_ref=p.s_ref)
    f, g = oracle.init(dom, np.ones(n ** 3), u0, s=s0)
    if dh is not None:
        f = f + dh
    if dg is not None:
        g = g + dg
    f, g = oracle.step(dom, op, f, g, n_steps=n_steps)
    _, _, s = oracle.macro(dom, op, f, g)
    return 0.5 * np.sum((s - target) ** 2)


def gpu_grads(p, u0, s0, theta, target, n_steps, every):
    n = N1
    lev = Level(n, n, n, p, scalar=True, force=np.zeros((3, n ** 3)))
    lev.init_equilibrium(np.ones(n ** 3), u0, s0)
    h0, g0 = lev.get_populations(shifted=True)
    th = torch.tensor(theta, dtype=torch.float32, device="cuda", requires_grad=True)
    h0 = h0.clone().requires_grad_(True)
    g0 = g0.clone().requires_grad_(True)
    s = rollout(lev, th, h0, g0, n_steps, every)
    tgt = torch.tensor(target, dtype=torch.float32, device="cuda")
    loss = 0.5 * ((s - tgt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (th.grad.double().cpu().numpy(), h0.grad.double().cpu().numpy(),
            g0.grad.double().cpu().numpy(), float(loss.detach()))


@pytest.mark.parametrize("adaptive", [True, False])
def test_gradients_match_fp64_finite_differences(adaptive):
    n_steps = 20
    p, u0, s0, theta, target = scene(adaptive=adaptive)
    gth, gh, gg, loss = gpu_grads(p, u0, s0, theta, target, n_steps, every=5)
    l0 = oracle_loss(p, u0, s0, theta, target, n_steps)
    assert loss == pytest.approx(l0, rel=1e-4)
    for k in range(3):
        v = inputs.smooth_random_field(N1, N1, N1, 1e-4, 60 + k, k_max=3)
        eps = 1e-3
        lp = oracle_loss(p, u0, s0, theta + eps * v, target, n_steps)
        lm = oracle_loss(p, u0, s0, theta - eps * v, target, n_steps)
        fd = (lp - lm) / (2 * eps)
        ad = float(np.sum(gth * v))
        assert ad == pytest.approx(fd, rel=1e-3), (k, ad, fd)
    # initial populations and scalar
    vh = 1e-5 * inputs.perturbation((27, N1 ** 3), 70)
    vg = 1e-4 * inputs.perturbation((7, N1 ** 3), 71)
    for dh, dg, gi in ((vh, None, gh), (None, vg, gg)):
        eps = 1e-2
        lp = oracle_loss(p, u0, s0, theta, target, n_steps,
                         None if dh is None else eps * dh, None if dg is None else eps * dg)
        lm = oracle_loss(p, u0, s0, theta, target, n_steps,
                         None if dh is None else -eps * dh, None if dg is None else -eps * dg)
        fd = (lp - lm) / (2 * eps)
        ad = float(np.sum(gi * (dh if dh is not None else dg)))
        assert ad == pytest.approx(fd, rel=1e-3)


def test_checkpoint_interval_does_not_change_gradients():
    p, u0, s0, theta, target = scene()
    a = gpu_grads(p, u0, s0, theta, target, 12, every=12)
    b = gpu_grads(p, u0, s0, theta, target, 12, every=5)
    c = gpu_grads(p, u0, s0, theta, target, 12, every=1)
    for x, y in ((a, b), (a, c)):
        for u, v in zip(x[:3], y[:3]):
            np.testing.assert_array_equal(u, v)


def test_backward_uses_the_force_of_its_own_forward_pass():
    """Two rollouts on one level (the second with another force field and
    gravity coefficient), then the backward pass of the first: its gradients
    equal those of a single rollout, and the level keeps the second
    rollout's force and parameters."""
    n = N1
    p, u0, s0, theta, target = scene()
    lev = Level(n, n, n, p, scalar=True, force=np.zeros((3, n ** 3)))
    lev.init_equilibrium(np.ones(n ** 3), u0, s0)
    h0, g0 = lev.get_populations(shifted=True)
    tgt = torch.tensor(target, dtype=torch.float32, device="cuda")

    def run(th_np, params):
        lev.set_params(params)
        th = torch.tensor(th_np, dtype=torch.float32, device="cuda", requires_grad=True)
        h = h0.clone().requires_grad_(True)
        g = g0.clone().requires_grad_(True)
        loss = 0.5 * ((rollout(lev, th, h, g, 8, 3) - tgt) ** 2).sum()
        return loss, th, h, g

    loss1, th1, h1, g1 = run(theta, p)
    other = Params(**{**p.__dict__, "beta": 3e-3})
    with torch.no_grad():
        run(-2.0 * theta, other)
    loss1.backward()
    torch.cuda.synchronize()
    assert lev.params.beta == other.beta
    force_after = lev.force.reshape(3, lev.plane)[:, : lev.n].double().cpu().numpy()
    np.testing.assert_array_equal(force_after, np.float32(-2.0 * theta).astype(np.float64))
    ref = gpu_grads(p, u0, s0, theta, target, 8, every=3)
    for got, want in zip((th1.grad, h1.grad, g1.grad), ref[:3]):
        np.testing.assert_array_equal(got.double().cpu().numpy(), want)


def test_zero_step_rollout_returns_the_scalar_and_its_gradient():
    n = N1
    p, u0, s0, theta, target = scene()
    lev = Level(n, n, n, p, scalar=True, force=np.zeros((3, n ** 3)))
    lev.init_equilibrium(np.ones(n ** 3), u0, s0)
    h0, g0 = lev.get_populations(shifted=True)
    th = torch.tensor(theta, dtype=torch.float32, device="cuda", requires_grad=True)
    h = h0.clone().requires_grad_(True)
    g = g0.clone().requires_grad_(True)
    s = rollout(lev, th, h, g, 0, 5)
    s.sum().backward()
    torch.cuda.synchronize()
    np.testing.assert_allclose(s.detach().double().cpu().numpy(), g0.double().cpu().numpy().sum(axis=0),
                               rtol=1e-6, atol=1e-6)
    assert float(th.grad.abs().max()) == 0.0 and float(h.grad.abs().max()) == 0.0
    np.testing.assert_array_equal(g.grad.cpu().numpy(), np.ones((7, n ** 3), np.float32))


def test_adjoint_over_the_fp64_trajectory_in_the_differentiable_config_regime():
    """The regime of the 128^3 differentiable smoke (nu = 1e-3, S = 1.988;
    adaptive on with g_max = 0.1; tau_s = 0.51; beta = 1e-4, s_ref = the
    initial mean), at 16^3 over 24 steps with the loss against a seeded
    target run.  The adjoint steps are chained over the oracle's FP64
    forward trajectory rounded to FP32, so the comparison with central
    differences of the FP64 oracle measures the adjoint itself, not the
    divergence of an FP32 forward trajectory from the FP64 one."""
    n, steps = N1, 24
    N = n ** 3
    s0 = inputs.gaussian_blob(n, n, n, (8, 8, 4), 1.0)
    p = Params(nu=1e-3, g_max=0.1, adaptive=True, tau_s=0.51, beta=1e-4, s_ref=float(s0.mean()))
    op = oracle.Params(nu=p.nu, g_max=p.g_max, adaptive=True, tau_s=p.tau_s, beta=p.beta,
                       s_ref=p.s_ref)
    u0 = inputs.smooth_random_field(n, n, n, 0.02, 81, k_max=2)
    theta = inputs.smooth_random_field(n, n, n, 1e-4, 82, k_max=2)
    theta_t = inputs.smooth_random_field(n, n, n, 1e-5, 83, k_max=3)
    f0, g0 = oracle.init(oracle.Domain(n, n, n), np.ones(N), u0, s=s0)

    def final_s(th, dh=None, dg=None):
        dom = oracle.Domain(n, n, n, theta=th)
        f, g = oracle.step(dom, op, f0 if dh is None else f0 + dh, g0 if dg is None else g0 + dg,
                           n_steps=steps)
        return oracle.macro(dom, op, f, g)[2]

    target = final_s(theta_t)

    def loss(th, dh=None, dg=None):
        return 0.5 * np.sum((final_s(th, dh, dg) - target) ** 2)

    dom = oracle.Domain(n, n, n, theta=theta)
    traj = [(f0, g0)]
    for _ in range(steps):
        traj.append(oracle.step(dom, op, *traj[-1]))
    s_end = oracle.macro(dom, op, *traj[-1])[2]

    lev = Level(n, n, n, p, scalar=True, force=theta)
    P = lev.plane

    def planes(x, rows):
        t = torch.zeros(rows, P, dtype=torch.float32, device="cuda")
        t[:, :N] = torch.tensor(np.asarray(x).reshape(rows, N), dtype=torch.float32, device="cuda")
        return t.reshape(-1)

    lam = torch.zeros(27 * P, dtype=torch.float32, device="cuda")
    lam2 = torch.zeros_like(lam)
    mu = planes(np.tile(s_end - target, (7, 1)), 7)
    mu2 = torch.zeros_like(mu)
    dth = torch.zeros(3 * P, dtype=torch.float32, device="cuda")
    for k in reversed(range(steps)):
        fk, gk = traj[k]
        lev.adjoint_step(planes(fk - W[:, None], 27), planes(gk, 7), lam, mu, lam2, mu2, dth)
        lam, lam2 = lam2, lam
        mu, mu2 = mu2, mu
    torch.cuda.synchronize()
    gth = dth.reshape(3, P)[:, :N].double().cpu().numpy()
    gh = lam.reshape(27, P)[:, :N].double().cpu().numpy()
    gg = mu.reshape(7, P)[:, :N].double().cpu().numpy()
    for k in range(3):
        v = inputs.smooth_random_field(n, n, n, 1e-4, 90 + k, k_max=3)
        eps = 1e-3
        fd = (loss(theta + eps * v) - loss(theta - eps * v)) / (2 * eps)
        ad = float(np.sum(gth * v))
        print(f"theta direction {k}: adjoint {ad:.6e}, central difference {fd:.6e}", flush=True)
        assert ad == pytest.approx(fd, rel=1e-3), (k, ad, fd)
    vh = 1e-5 * inputs.perturbation((27, N), 95)
    vg = 1e-4 * inputs.perturbation((7, N), 96)
    for name, dh, dg, gi in (("f0", vh, None, gh), ("g0", None, vg, gg)):
        eps = 1e-2
        fd = (loss(theta, None if dh is None else eps * dh, None if dg is None else eps * dg)
              - loss(theta, None if dh is None else -eps * dh, None if dg is None else -eps * dg)) / (2 * eps)
        ad = float(np.sum(gi * (dh if dh is not None else dg)))
        print(f"{name} direction: adjoint {ad:.6e}, central difference {fd:.6e}", flush=True)
        assert ad == pytest.approx(fd, rel=1e-3)
