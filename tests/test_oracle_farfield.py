"""Pins of the oracle's far-field scales (spacing larger than the reference
scale; sections "Temporal alignment and scale mapping" and "Handling
multiple scales", reversed rules) and of the Neumann far-field boundary
(section "Initialization and boundary treatment")."""
import numpy as np
import pytest

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import inputs

from lbm_textbook import feq_second_order

C = oracle.velocities().astype(float)
W = oracle.weights()


def test_neumann_cells_copy_the_inward_neighbour():
    """Every NEUMANN cell's new state is the old state of the cell one step
    inward along each non-periodic face it lies on (faces, edges, corners);
    on a periodic axis nothing moves."""
    nx, ny, nz = 5, 4, 3
    n = nx * ny * nz
    x, y, z = inputs.grid_coords(nx, ny, nz)
    for periodic in (0, 4):
        face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1)
        if not periodic & 4:
            face |= (z == 0) | (z == nz - 1)
        flags = np.where(face, oracle.NEUMANN, oracle.FLUID).astype(np.uint8)
        f = 0.02 + inputs.perturbation((27, n), 11, 0.01)
        g = 0.1 + inputs.perturbation((7, n), 12, 0.01)
        dom = oracle.Domain(nx, ny, nz, periodic=periodic, flags=flags)
        fo, go = oracle.step(dom, oracle.Params(nu=0.01, g_max=0.1), f, g)
        for c in np.flatnonzero(face):
            xs = min(max(x[c], 1), nx - 2)
            ys = min(max(y[c], 1), ny - 2)
            zs = z[c] if periodic & 4 else min(max(z[c], 1), nz - 2)
            src = xs + nx * (ys + ny * zs)
            np.testing.assert_array_equal(fo[:, c], f[:, src])
            np.testing.assert_array_equal(go[:, c], g[:, src])


def window_scale(nx, ny, nz, origin, nu, shell_axes=7, periodic=0, f=None):
    """The reference scale as a window: GHOST shell on the faces of the
    listed axes (written from the far-field scale), FLUID inside."""
    x, y, z = inputs.grid_coords(nx, ny, nz)
    shell = np.zeros(x.size, bool)
    for a, (c, m) in enumerate(((x, nx), (y, ny), (z, nz))):
        if shell_axes & (1 << a):
            shell |= (c == 0) | (c == m - 1)
    fl = np.where(shell, oracle.GHOST, oracle.FLUID).astype(np.uint8)
    return ml.OScale(nx, ny, nz, 1.0, origin, oracle.Params(nu=nu, g_max=0.05), fl,
                     periodic=periodic, f=f)


def far_field_scale(nx, ny, nz, dx, origin, nu, window: ml.OScale, periodic=0, f=None):
    """A coarser scale around `window`: its cells whose trilinear stencil in
    the window consists of FLUID cells are GHOST (mapped from the window);
    its faces on non-periodic axes are NEUMANN."""
    x, y, z = inputs.grid_coords(nx, ny, nz)
    fl = np.full(x.size, oracle.FLUID, np.uint8)
    probe = ml.OScale(nx, ny, nz, dx, origin, oracle.Params(nu=nu), fl.copy(), periodic=periodic)
    overlap = ml.post_targets(probe, window)
    fl[overlap] = oracle.GHOST
    for a, (c, m) in enumerate(((x, nx), (y, ny), (z, nz))):
        if not periodic & (1 << a):
            fl[(c == 0) | (c == m - 1)] = oracle.NEUMANN
    return ml.OScale(nx, ny, nz, dx, origin, oracle.Params(nu=nu, g_max=0.05), fl,
                     periodic=periodic, parent=0, f=f)


def test_far_field_scale_with_the_reference_spacing_reproduces_the_single_scale_run():
    """A far-field scale whose spacing exceeds the reference's by 1e-12
    (alpha_c -> 1, nodes coincide to 1e-11) around a reference window: after
    4 reference steps the window and the far field both equal the
    single-scale run on the whole periodic box."""
    n = 16
    nu = 0.01
    rho, u = inputs.taylor_green_3d(n, 0.04)
    dom = oracle.Domain(n, n, n)
    f0, _ = oracle.init(dom, rho, u)
    ref, _ = oracle.step(dom, oracle.Params(nu=nu, g_max=0.05), f0, n_steps=4)
    o = (4, 5, 3)
    wn = (8, 7, 9)
    idx = np.array([(xx + o[0]) + n * ((yy + o[1]) + n * (zz + o[2]))
                    for zz in range(wn[2]) for yy in range(wn[1]) for xx in range(wn[0])])
    s0 = window_scale(*wn, tuple(float(v) for v in o), nu, f=f0[:, idx].copy())
    eps = 1e-12
    ff = far_field_scale(n, n, n, 1.0 + eps, (0.0, 0.0, 0.0), nu / (1.0 + eps), s0, periodic=7,
                         f=f0.copy())
    scales = [s0, ff]
    ml.prepare(scales)
    assert ff.ghosts.size > 0 and ff.post[0].size == np.count_nonzero(s0.flags == oracle.GHOST)
    ml.multiscale_step(scales, 4)
    np.testing.assert_allclose(s0.f, ref[:, idx], rtol=0, atol=1e-9)
    np.testing.assert_allclose(ff.f, ref, rtol=0, atol=1e-9)


@pytest.mark.parametrize("dx_c", [2.0, 1 / 0.75])
def test_uniform_flow_stays_uniform_with_a_far_field_scale(dx_c):
    u0 = np.array([0.03, -0.01, 0.02])
    feq = feq_second_order(1.0, u0, C, W)
    nu0 = 1e-3
    wn = (9, 8, 8)
    s0 = window_scale(*wn, (6.0, 5.0, 5.0), nu0)
    s0.f = np.tile(feq[:, None], (1, s0.n))
    nc = 14
    ff = far_field_scale(nc, nc, nc, dx_c, (0.0, 0.0, 0.0), nu0 / dx_c, s0)
    ff.f = np.tile(feq[:, None], (1, ff.n))
    scales = [s0, ff]
    ml.prepare(scales)
    ml.multiscale_step(scales, 3)
    for s in scales:
        np.testing.assert_allclose(s.f, np.tile(feq[:, None], (1, s.n)), rtol=0, atol=1e-14)


def test_taylor_green_window_inside_a_far_field_scale_keeps_the_closed_form_decay():
    """2D Taylor-Green vortex of wavelength 64 on a periodic far-field scale
    of spacing 2 (alpha_c = 0.5), with a reference window of spacing 1 over
    the central 32 x 32 (periodic in z): after 100 reference steps the
    window's mode amplitude is within 1 % of exp(-2 nu k^2 t)."""
    L = 64
    nu0 = 0.1 / 3.0
    k = 2 * np.pi / L
    u0 = 0.05

    def tgv(px, py):
        u = np.zeros((3, px.size))
        u[0] = u0 * np.cos(k * px) * np.sin(k * py)
        u[1] = -u0 * np.sin(k * px) * np.cos(k * py)
        return u

    wn = (33, 33, 4)
    o = (16.0, 16.0, 0.0)
    xs, ys, zs = inputs.grid_coords(*wn)
    uw = tgv(o[0] + xs, o[1] + ys)
    s0 = window_scale(*wn, o, nu0, shell_axes=3, periodic=4)
    s0.f, _ = oracle.init(oracle.Domain(*wn), np.ones(s0.n), uw)
    dxc = 2.0
    nc = (32, 32, 2)
    xc, yc, _ = inputs.grid_coords(*nc)
    uc = tgv(xc * dxc, yc * dxc)
    ff = far_field_scale(*nc, dxc, (0.0, 0.0, 0.0), nu0 / dxc, s0, periodic=7)
    ff.f, _ = oracle.init(oracle.Domain(*nc), np.ones(ff.n), uc)
    scales = [s0, ff]
    ml.prepare(scales)
    steps = 100
    ml.multiscale_step(scales, steps)
    _, us, _ = oracle.macro(s0.domain(), s0.params, s0.f)
    inner = s0.flags == oracle.FLUID
    amp = np.sum(us[:2, inner] * uw[:2, inner]) / np.sum(uw[:2, inner] ** 2)
    exact = np.exp(-2.0 * nu0 * k * k * steps)
    assert amp == pytest.approx(exact, rel=1e-2)
