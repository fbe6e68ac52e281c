"""Pins of the oracle's finite-difference gradient variant of the adaptive
relaxation (section "Adaptive relaxation": the factor follows |grad u|):
the gradient field against closed forms, and the step in that mode against
stream + per-cell collision with the given gradient."""
import numpy as np
import pytest

import oracle
from paper_1807_02284_amd import inputs

W = oracle.weights()


def equilibrium_state(nx, ny, nz, u, periodic=7):
    dom = oracle.Domain(nx, ny, nz, periodic=periodic,
                        flags=None if periodic == 7 else np.zeros(nx * ny * nz, np.uint8))
    f, _ = oracle.init(dom, np.ones(nx * ny * nz), u)
    return dom, f


def test_grad_field_of_a_shear_wave_is_the_central_difference():
    nx, ny, nz = 4, 24, 3
    U = 0.03
    k = 2 * np.pi / ny
    _, y, _ = inputs.grid_coords(nx, ny, nz)
    u = np.zeros((3, y.size))
    u[0] = U * np.sin(k * y)
    dom, f = equilibrium_state(nx, ny, nz, u)
    G = oracle.grad_field(dom, oracle.Params(), f)
    np.testing.assert_allclose(G, np.abs(U * np.sin(k) * np.cos(k * y)), rtol=0, atol=1e-14)


def test_grad_field_of_a_linear_field_is_its_frobenius_norm_everywhere():
    """u = A x on a non-periodic box: central differences inside and
    one-sided differences on the faces are all exact."""
    nx, ny, nz = 6, 5, 7
    A = np.array([[0.001, -0.002, 0.0005], [0.0015, 0.0, -0.001], [-0.0007, 0.0012, 0.002]])
    x, y, z = inputs.grid_coords(nx, ny, nz)
    X = np.stack([x, y, z]).astype(float)
    u = A @ X - (A @ X).mean(axis=1, keepdims=True)
    dom, f = equilibrium_state(nx, ny, nz, u, periodic=0)
    G = oracle.grad_field(dom, oracle.Params(), f)
    np.testing.assert_allclose(G, np.sqrt(np.sum(A * A)), rtol=1e-10, atol=0)


def test_collide_with_its_own_gradient_estimate_equals_collide():
    rng = np.random.default_rng(3)
    p = oracle.Params(nu=0.01, g_max=0.05)
    u = np.array([0.02, -0.01, 0.015])
    f = oracle.equilibrium(1.01, u) + 1e-4 * W * rng.standard_normal(27)
    out, diag = oracle.collide(f, p)
    out_g, diag_g = oracle.collide_g(f, p, diag["G"])
    np.testing.assert_array_equal(out_g, out)
    assert diag_g["phi"] == diag["phi"]


def test_gradient_mode_step_is_stream_then_collide_with_the_lagged_gradient():
    """The step in gradient mode equals: G from the stored (pre-stream)
    velocity field, then pull-stream, then the per-cell collision with that
    G; the force and the scalar are included."""
    nx, ny, nz = 7, 6, 5
    n = nx * ny * nz
    u = inputs.smooth_random_field(nx, ny, nz, 0.04, 5, k_max=2)
    s = 0.5 + 0.2 * inputs.smooth_random_field(nx, ny, nz, 1.0, 6, k_max=1)[0]
    theta = inputs.smooth_random_field(nx, ny, nz, 1e-4, 7, k_max=1)
    dom = oracle.Domain(nx, ny, nz, theta=theta)
    p = oracle.Params(nu=0.005, g_max=0.02, tau_s=0.6, beta=1e-3, s_ref=0.5, grad_mode=1)
    f, g = oracle.init(dom, np.ones(n), u, s=s)
    f = f + 1e-4 * W[:, None] * inputs.perturbation((27, n), 8)
    G = oracle.grad_field(dom, p, f, g)
    assert np.all(G > 0) and np.any(G > p.g_max) and np.any(G < p.g_max)
    fs, gs = oracle.stream(dom, f, g)
    expect = np.zeros_like(f)
    for c in range(n):
        sc = gs[:, c].sum()
        F = theta[:, c].copy()
        F[2] += p.beta * (sc - p.s_ref)
        expect[:, c], _ = oracle.collide_g(fs[:, c], p, G[c], F)
    got, _ = oracle.step(dom, p, f, g)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-15)
    # and the local mode differs (the two estimates are not the same field)
    local, _ = oracle.step(dom, oracle.Params(**{**p.__dict__, "grad_mode": 0}), f, g)
    assert np.max(np.abs(local - got)) > 1e-9


def test_gradient_modes_agree_on_uniform_flow():
    nx = ny = nz = 6
    u = np.tile(np.array([[0.02], [-0.01], [0.03]]), (1, nx * ny * nz))
    dom, f = equilibrium_state(nx, ny, nz, u)
    a, _ = oracle.step(dom, oracle.Params(nu=0.01, grad_mode=0), f, n_steps=3)
    b, _ = oracle.step(dom, oracle.Params(nu=0.01, grad_mode=1), f, n_steps=3)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_running_maximum_normalises_by_the_fields_largest_gradient():
    """With gmax_running the step equals the step with g_max set to the
    maximum of the gradient field, so no cell is clamped and the cell with
    the largest gradient gets the smallest factor a + b."""
    nx, ny, nz = 9, 8, 6
    n = nx * ny * nz
    u = inputs.smooth_random_field(nx, ny, nz, 0.05, 15, k_max=2)
    dom = oracle.Domain(nx, ny, nz)
    f, _ = oracle.init(dom, np.ones(n), u)
    p = oracle.Params(nu=0.005, g_max=1e-9, grad_mode=1, gmax_running=True)
    G = oracle.grad_field(dom, p, f)
    fixed = oracle.Params(**{**p.__dict__, "gmax_running": False, "g_max": float(G.max())})
    a, _ = oracle.step(dom, p, f)
    b, _ = oracle.step(dom, fixed, f)
    np.testing.assert_array_equal(a, b)
    # the tiny constant g_max would clamp every cell instead
    c, _ = oracle.step(dom, oracle.Params(**{**p.__dict__, "gmax_running": False}), f)
    assert np.max(np.abs(c - a)) > 1e-9
    fs, _ = oracle.stream(dom, f)
    k = int(np.argmax(G))
    _, diag = oracle.collide_g(fs[:, k], fixed, G[k])
    assert diag["phi"] == pytest.approx(fixed.a + fixed.b)
