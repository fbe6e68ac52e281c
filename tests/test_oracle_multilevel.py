"""Pins of the oracle's cross-scale exchange, temporal interpolation and
multi-scale scheduler (sections "Mapping distribution functions" to
"Handling multiple scales", Algorithm 1)."""
import math

import numpy as np
import pytest

import oracle
from lbm_textbook import feq_second_order
from oracle import multilevel as ml
from paper_1807_02284_amd import inputs

C = oracle.velocities().astype(float)
W = oracle.weights()
CS = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
WS = np.array([0.25] + [0.125] * 6)


def geom(nx, ny, nz, origin, dx, nu, periodic=0, tau_s=0.0):
    return dict(nx=nx, ny=ny, nz=nz, periodic=periodic, origin=origin, dx=dx, nu=nu, tau_s=tau_s)


def test_time_interp_exact_for_quadratics_and_nodes():
    t = (0.0, 2.0 / 3.0, 4.0 / 3.0)
    a, b, c = inputs.perturbation((3, 50), 1)
    s = [a + b * ti + c * ti * ti for ti in t]
    for te in (1.0, 0.3, 4.0 / 3.0):
        np.testing.assert_allclose(oracle.time_interp(*s, t, te), a + b * te + c * te * te,
                                   rtol=0, atol=1e-14)
    np.testing.assert_allclose(oracle.time_interp(*s, t, t[1]), s[1], rtol=0, atol=1e-15)


def test_exchange_is_identity_on_coincident_lattices_with_equal_rates():
    src = geom(6, 5, 4, (0.0, 0.0, 0.0), 1.0, 0.01)
    dst = geom(3, 3, 2, (2.0, 1.0, 1.0), 1.0, 0.01)
    f = W[:, None] * (1.0 + 0.05 * inputs.perturbation((27, 120), 2))
    out = np.zeros(27 * 18)
    cells = np.arange(18)
    oracle.exchange(src, f, f, 0.0, dst, cells, out)
    out = out.reshape(27, 18)
    for c in cells:
        x, y, z = c % 3 + 2, (c // 3) % 3 + 1, c // 9 + 1
        np.testing.assert_allclose(out[:, c], f[:, x + 6 * (y + 5 * z)], rtol=0, atol=1e-15)


def test_exchange_returns_trilinear_interpolant_when_rates_agree():
    """alpha = 1, equal rates: K^ = I and the mapping returns the trilinear
    interpolant, which is exact for fields linear in space."""
    nx, ny, nz = 6, 5, 4
    src = geom(nx, ny, nz, (0.0, 0.0, 0.0), 1.0, 0.02)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    a = W * (1 + 0.1 * inputs.perturbation(27, 3))
    b = 1e-3 * W[:, None] * inputs.perturbation((27, 3), 4)
    f = a[:, None] + b[:, 0:1] * x + b[:, 1:2] * y + b[:, 2:3] * z
    dst = geom(3, 2, 2, (1.3, 0.6, 1.45), 1.0, 0.02)
    out = np.zeros(27 * 12)
    oracle.exchange(src, f, f, 0.0, dst, np.arange(12), out)
    out = out.reshape(27, 12)
    dx_, dy_, dz_ = inputs.grid_coords(3, 2, 2)
    for c in range(12):
        p = (1.3 + dx_[c], 0.6 + dy_[c], 1.45 + dz_[c])
        np.testing.assert_allclose(out[:, c], a + b[:, 0] * p[0] + b[:, 1] * p[1] + b[:, 2] * p[2],
                                   rtol=0, atol=1e-15)


@pytest.mark.parametrize("ratio", [1.5, 2.0, 1.0 / 1.5])
def test_uniform_flow_is_invariant_under_exchange(ratio):
    rho, u = 1.02, np.array([0.04, -0.03, 0.02])
    feq = feq_second_order(rho, u, C, W)
    src = geom(8, 8, 8, (0.0, 0.0, 0.0), 1.0, 1e-3)
    f = np.tile(feq[:, None], (1, 512))
    n = 3 * 3 * 3
    dst = geom(3, 3, 3, (2.2, 1.7, 3.1), 1.0 / ratio, 1e-3 * ratio)
    out = np.zeros(27 * n)
    oracle.exchange(src, f, f, 0.0, dst, np.arange(n), out)
    np.testing.assert_allclose(out.reshape(27, n), np.tile(feq[:, None], (1, n)), rtol=0, atol=1e-15)


def chapman_enskog_post(rho, u, grad_u, S):
    """Post-collision state of a steady linear flow in lattice units:
    f~ = f^eq + (1 - S) w_i/(2 cs^4) Q_i : Pi, Pi = -2 cs^2 rho S^ / S
    (eq. epsilon_f1, eq. pi_1)."""
    cs2 = 1.0 / 3.0
    Shat = 0.5 * (grad_u + grad_u.T)
    Pi = -2.0 * cs2 * rho * Shat / S
    Q = np.einsum("ia,ib->iab", C, C) - cs2 * np.eye(3)[None]
    return feq_second_order(rho, u, C, W) + (1.0 - S) * W / (2 * cs2 * cs2) * np.einsum("iab,ab->i", Q, Pi)


@pytest.mark.parametrize("alpha", [2.0, 1.5, 0.5])
def test_exchange_rescales_nonequilibrium_like_a_resolved_shear(alpha):
    """A steady linear shear mapped from one scale to another, at points that
    coincide with source nodes: the stress moments m4..m8, density and
    momentum equal those of the Chapman-Enskog state the target scale itself
    would hold for the same physical flow (velocity identical in lattice
    units, velocity gradient scaled with the spacing, viscosity scaled by
    alpha).  The non-equilibrium parts of m9..m26 are carried over unscaled
    (the unit entries of K)."""
    nu_s = 0.002
    dx_s, dx_d = 1.0, 1.0 / alpha
    nu_d = nu_s * alpha
    S_s, S_d = 1 / (3 * nu_s + 0.5), 1 / (3 * nu_d + 0.5)
    G = np.array([[0.0, 2e-3, 0.0], [0.0, 0.0, -1e-3], [1.5e-3, 0.0, 0.0]])  # physical du_a/dx_b
    G -= np.trace(G) / 3 * np.eye(3)
    u0 = np.array([0.03, -0.01, 0.02])
    n = 6
    src = geom(n, n, n, (0.0, 0.0, 0.0), dx_s, nu_s)
    xs, ys, zs = inputs.grid_coords(n, n, n)
    f = np.zeros((27, n ** 3))
    for c in range(n ** 3):
        p = np.array([xs[c], ys[c], zs[c]]) * dx_s
        f[:, c] = chapman_enskog_post(1.0, u0 + G @ p, G * dx_s, S_s)
    # source nodes that are also target nodes for alpha in {2, 1.5, 0.5}
    pts = [np.array([a, b, c_], float) for a in (2, 4) for b in (2, 4) for c_ in (2, 4)]
    dst = geom(8, 8, 8, (2.0, 2.0, 2.0), dx_d, nu_d)
    cells = []
    for p in pts:
        q = np.rint((p - 2.0) / dx_d).astype(int)
        assert np.allclose(q * dx_d + 2.0, p)
        cells.append(q[0] + 8 * (q[1] + 8 * q[2]))
    out = np.zeros(27 * 512)
    oracle.exchange(src, f, f, 0.0, dst, np.array(cells), out)
    out = out.reshape(27, 512)
    for p, c in zip(pts, cells):
        u = u0 + G @ p
        expect = chapman_enskog_post(1.0, u, G * dx_d, S_d)
        M = oracle.basis(u)
        meq = oracle.meq(1.0, u)
        np.testing.assert_allclose((M.T @ out[:, c])[:9], (M.T @ expect)[:9], rtol=0, atol=1e-15)
        src_c = int(round(p[0])) + n * (int(round(p[1])) + n * int(round(p[2])))
        np.testing.assert_allclose((M.T @ out[:, c])[9:] - meq[9:], (M.T @ f[:, src_c])[9:] - meq[9:],
                                   rtol=0, atol=1e-15)


def test_scalar_exchange_rescales_gradient_part():
    """Linear scalar at rest: post-collision g~ = g^eq(s) - (tau - 1) w_i c_i .
    grad s dx; mapping to a scale with tau' - 1/2 = alpha (tau - 1/2) gives
    the target scale's own state for the same physical gradient."""
    alpha, tau = 2.0, 0.6
    tau_d = 0.5 + alpha * (tau - 0.5)
    sg = np.array([0.01, -0.02, 0.005])
    n = 5
    src = geom(n, n, n, (0.0, 0.0, 0.0), 1.0, 0.01, tau_s=tau)
    dst = geom(4, 4, 4, (2.0, 2.0, 2.0), 1.0 / alpha, 0.02, tau_s=tau_d)
    xs, ys, zs = inputs.grid_coords(n, n, n)
    feq = np.tile(W[:, None], (1, n ** 3))
    g = np.zeros((7, n ** 3))
    for c in range(n ** 3):
        s = 0.5 + sg @ np.array([xs[c], ys[c], zs[c]])
        g[:, c] = WS * s - (tau - 1.0) * WS * (CS @ sg)
    cell = 0 + 4 * (0 + 4 * 0)       # target point (2, 2, 2) = a source node
    fo = np.zeros(27 * 64)
    go = np.zeros(7 * 64)
    oracle.exchange(src, feq, feq, 0.0, dst, np.array([cell]), fo, g, g, go)
    s = 0.5 + sg @ np.array([2.0, 2.0, 2.0])
    expect = WS * s - (tau_d - 1.0) * WS * (CS @ sg) / alpha
    np.testing.assert_allclose(go.reshape(7, 64)[:, cell], expect, rtol=0, atol=1e-15)


def box_scale(nx, ny, nz, origin, dx, nu, f=None):
    fl = np.zeros(nx * ny * nz, dtype=np.uint8)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    shell = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    fl[shell] = oracle.GHOST
    return ml.OScale(nx, ny, nz, dx, origin, oracle.Params(nu=nu, g_max=0.05), fl,
                     periodic=0, parent=0, f=f)


def test_alpha_one_two_scale_run_equals_single_scale_run():
    """A finer scale with the reference spacing on coincident lattice points
    (K^ = I, trilinear at nodes): every scale reproduces the single-scale
    solution (l = 2 sub-steps, quadratic time interpolation hits the node)."""
    n = 12
    nu = 0.01
    rho, u = inputs.taylor_green_3d(n, 0.04)
    dom = oracle.Domain(n, n, n)
    f0, _ = oracle.init(dom, rho, u)
    ref, _ = oracle.step(dom, oracle.Params(nu=nu, g_max=0.05), f0, n_steps=3)
    s0 = ml.OScale(n, n, n, 1.0, (0.0, 0.0, 0.0), oracle.Params(nu=nu, g_max=0.05),
                   np.zeros(n ** 3, np.uint8), periodic=7, f=f0.copy())
    fine = box_scale(6, 7, 5, (3.0, 2.0, 4.0), 1.0, nu)
    idx = [(x + 3) + n * ((y + 2) + n * (z + 4)) for z in range(5) for y in range(7) for x in range(6)]
    fine.f = f0[:, idx].copy()
    scales = [s0, fine]
    ml.prepare(scales)
    assert fine.post[0].size == 4 * 5 * 3
    ml.multiscale_step(scales, 3)
    np.testing.assert_allclose(scales[0].f, ref, rtol=0, atol=1e-14)
    inner = np.flatnonzero(fine.flags == oracle.FLUID)
    np.testing.assert_allclose(fine.f[:, inner], ref[:, np.array(idx)[inner]], rtol=0, atol=1e-14)


def test_uniform_flow_stays_uniform_on_three_scales():
    n = 12
    rho, u = 1.0, np.array([0.03, 0.01, -0.02])
    feq = feq_second_order(rho, u, C, W)
    nu0 = 1e-3
    s0 = ml.OScale(n, n, n, 1.0, (0.0, 0.0, 0.0), oracle.Params(nu=nu0, g_max=0.05),
                   np.zeros(n ** 3, np.uint8), periodic=7, f=np.tile(feq[:, None], (1, n ** 3)))
    s1 = box_scale(10, 9, 9, (2.3, 2.6, 2.2), 1 / 1.5, nu0 * 1.5)
    s1.f = np.tile(feq[:, None], (1, s1.n))
    s2 = box_scale(8, 7, 7, (3.4, 3.6, 3.3), 0.5, nu0 * 2.0)
    s2.parent = 1
    s2.f = np.tile(feq[:, None], (1, s2.n))
    scales = [s0, s1, s2]
    ml.prepare(scales)
    assert s2.post[0].size > 0 and s2.post[1].size > 0
    ml.multiscale_step(scales, 2)
    for s in scales:
        np.testing.assert_allclose(s.f, np.tile(feq[:, None], (1, s.n)), rtol=0, atol=1e-14)


def test_two_scale_taylor_green_keeps_closed_form_decay():
    """2D Taylor-Green on a 32^2 reference lattice with an alpha = 1.5 patch
    covering the centre: the mode amplitude after 100 reference steps stays
    within 2 % of the single-scale run (interpolation adds a little diffusion)."""
    n, nz = 32, 2
    tau = 0.6
    nu0 = (tau - 0.5) / 3
    rho, u = inputs.taylor_green_2d(n, n, nz, 0.05)
    dom = oracle.Domain(n, n, nz)
    f0, _ = oracle.init(dom, rho, u)
    single, _ = oracle.step(dom, oracle.Params(nu=nu0, g_max=0.1), f0, n_steps=100)
    _, us, _ = oracle.macro(dom, oracle.Params(nu=nu0), single)
    s0 = ml.OScale(n, n, nz, 1.0, (0.0, 0.0, 0.0), oracle.Params(nu=nu0, g_max=0.1),
                   np.zeros(n * n * nz, np.uint8), periodic=7, f=f0.copy())
    # fine patch: 1.5x resolution over [8, 24]^2, periodic in z (nz fine = 3)
    alpha = 1.5
    nf = 25
    fine = box_scale(nf, nf, 3, (8.0, 8.0, 0.0), 1 / alpha, nu0 * alpha)
    fine.periodic = 4
    xs, ys, zs = inputs.grid_coords(nf, nf, 3)
    fine.flags[:] = oracle.FLUID
    fine.flags[(xs == 0) | (xs == nf - 1) | (ys == 0) | (ys == nf - 1)] = oracle.GHOST
    k = 2 * np.pi / n
    px, py = 8.0 + xs / alpha, 8.0 + ys / alpha
    uf = np.zeros((3, fine.n))
    uf[0] = 0.05 * np.cos(k * px) * np.sin(k * py)
    uf[1] = -0.05 * np.sin(k * px) * np.cos(k * py)
    fine.f, _ = oracle.init(oracle.Domain(nf, nf, 3), np.ones(fine.n), uf)
    scales = [s0, fine]
    ml.prepare(scales)
    ml.multiscale_step(scales, 100)
    _, um, _ = oracle.macro(dom, oracle.Params(nu=nu0), scales[0].f)
    amp_single = (us[0] * u[0]).sum() / (u[0] * u[0]).sum()
    amp_multi = (um[0] * u[0]).sum() / (u[0] * u[0]).sum()
    assert amp_multi == pytest.approx(amp_single, rel=0.02)


@pytest.mark.parametrize("alpha", [1.5, 2.0, 2.5])
def test_shell_before_each_substep_holds_the_parent_state_at_its_time(alpha, monkeypatch):
    """Section "Temporal alignment and scale mapping": before each of the
    first l - 1 sub-steps the finer scale's boundary is mapped from the
    parent blended between t_n and t_n + dt_0 (read here at the sub-step's
    start time, (k - 1) dt_f), and before the final sub-step directly from
    the parent at t_n + dt_0.  A uniform periodic parent under a uniform body
    force F has the closed-form post-collision momentum j(t_n + t dt_0) =
    j(t_n) + t F (momentum rises by exactly F per step, linear in time), and
    the mapping keeps density and momentum, so the shell's momentum before
    each sub-step names the parent time it was mapped from."""
    n = 8
    F0 = np.array([2e-4, -1e-4, 5e-5])
    u0 = np.array([0.02, 0.01, -0.01])
    feq = feq_second_order(1.0, u0, C, W)
    s0 = ml.OScale(n, n, n, 1.0, (0.0, 0.0, 0.0), oracle.Params(nu=1e-3, g_max=0.05),
                   np.zeros(n ** 3, np.uint8), periodic=7, f=np.tile(feq[:, None], (1, n ** 3)),
                   theta=np.tile(F0[:, None], (1, n ** 3)))
    nf = 6
    fine = box_scale(nf, nf, nf, (2.2, 2.1, 2.3), 1 / alpha, 1e-3 * alpha)
    fine.f = np.tile(feq[:, None], (1, fine.n))
    fine.theta = np.tile((F0 / alpha)[:, None], (1, fine.n))
    scales = [s0, fine]
    ml.prepare(scales)
    j0 = C.T @ s0.f[:, 0]
    seen = []
    real_step = ml.step

    def spy(dom, params, f, g=None, n_steps=1):
        if dom.n == fine.n:
            seen.append(np.asarray(f).reshape(27, fine.n)[:, fine.ghosts].copy())
        return real_step(dom, params, f, g, n_steps)

    monkeypatch.setattr(ml, "step", spy)
    ml.multiscale_step(scales, 1)
    l = math.floor(alpha) + 1
    assert len(seen) == l
    for k, shell in enumerate(seen, start=1):
        t = 1.0 if k == l else (k - 1) / alpha
        np.testing.assert_allclose(C.T @ shell, np.tile((j0 + t * F0)[:, None], (1, shell.shape[1])),
                                   rtol=0, atol=2e-15)
    # the parent itself, outside the cells post-mapped from the finer
    # scale: exactly F more momentum after the reference step
    out = np.setdiff1d(np.arange(n ** 3), fine.post[0])
    assert 0 < out.size < n ** 3
    np.testing.assert_allclose(C.T @ scales[0].f[:, out], np.tile((j0 + F0)[:, None], (1, out.size)),
                               rtol=0, atol=2e-15)
