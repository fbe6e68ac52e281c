"""Pins of the oracle's no-slip wall node (kind WALL): the second-order wall
treatment that section "Initialization and boundary treatment" takes from
Latt et al., written as the regularized boundary condition of Latt &
Chopard (Math. Comput. Simul. 72, 2006; Latt, Chopard, Malaspinas, Deville
and Michler, Phys. Rev. E 77, 056703, 2008) for a flat wall through the node.
The paper prints no formula for it, so its parity with the paper is unpinned;
these tests pin the oracle to the method's own closed forms."""
import numpy as np
import pytest

import oracle
from lbm_textbook import feq_second_order
from paper_1807_02284_amd import inputs

C = oracle.velocities().astype(float)
W = oracle.weights()
NORMALS = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def regularized_state(rho, u, Pi):
    """f^eq(rho, u) + w_i / (2 cs^4) (c_i c_i - cs^2 I) : Pi (textbook
    second-order Hermite state with non-equilibrium stress Pi)."""
    Q = np.einsum("ia,ib->iab", C, C) - np.eye(3)[None] / 3.0
    return feq_second_order(rho, u, C, W) + 4.5 * W * np.einsum("iab,ab->i", Q, Pi)


@pytest.mark.parametrize("n", NORMALS)
def test_regularization_returns_a_regularized_state_whatever_comes_from_the_wall(n):
    """A node whose known populations (c.n >= 0) belong to a regularized
    state with wall velocity zero, f^eq(rho, -F/(2 rho)) + Hermite stress
    part, gets exactly that state back, whatever the unknown populations
    (c.n < 0, pulled from the wall) hold: density from mass and normal
    momentum, stress from the bounced non-equilibrium, reconstruction."""
    rng = np.random.default_rng(7 + sum((k + 2) * 3 ** a for a, k in enumerate(n)))
    unknown = C @ np.array(n, float) < 0
    assert unknown.sum() == 9
    for _ in range(5):
        rho = 1.0 + 0.05 * rng.uniform(-1, 1)
        F = 1e-4 * rng.uniform(-1, 1, 3)
        A = 1e-3 * rng.uniform(-1, 1, (3, 3))
        Pi = A + A.T
        S = regularized_state(rho, -F / (2 * rho), Pi)
        f = S.copy()
        f[unknown] = rng.uniform(0.0, 0.1, unknown.sum())
        out = oracle.wall_regularize(f, n, F)
        np.testing.assert_allclose(out, S, rtol=0, atol=1e-15)
        # density and momentum of the result: rho and -F/2 (wall velocity 0)
        assert out.sum() == pytest.approx(rho, abs=1e-15)
        np.testing.assert_allclose(C.T @ out, -F / 2, rtol=0, atol=1e-16)


def channel(N, nu, F, steps, wall_kind):
    """Force-driven flow between two walls normal to y, periodic in x and
    z (1 x N x 1 lattice).  WALL: wall nodes at y = 0 and y = N - 1, the
    walls through them; SOLID: halfway bounce-back, the walls at y = 0.5
    and y = N - 1.5."""
    fl = np.zeros(N, np.uint8)
    fl[0] = fl[-1] = wall_kind
    th = np.zeros((3, N))
    th[0] = F
    dom = oracle.Domain(1, N, 1, periodic=5, flags=fl, theta=th)
    p = oracle.Params(nu=nu, g_max=0.1)
    f, _ = oracle.init(dom, np.ones(N), np.zeros((3, N)))
    f, _ = oracle.step(dom, p, f, n_steps=steps)
    return oracle.macro(dom, p, f)


def test_force_driven_channel_converges_at_second_order_to_the_parabola_through_the_wall_nodes():
    """Closed form u(y) = F/(2 nu) y (H - y) with the walls on the node planes
    y = 0 and y = H = N - 1: the wall nodes hold u = 0 exactly, and the
    largest error relative to the centre-line speed falls by 4 when the
    resolution doubles (N = 9 -> 17 -> 33 at fixed nu, steady state)."""
    nu, F = 0.3, 1e-6
    errs = []
    for N in (9, 17, 33):
        H = N - 1
        rho, u, _ = channel(N, nu, F, int(8 * H * H / nu) + 200, oracle.WALL)
        y = np.arange(N, dtype=float)
        exact = F / (2 * nu) * y * (H - y)
        assert abs(u[0, 0]) <= 1e-15 and abs(u[0, -1]) <= 1e-15
        np.testing.assert_allclose(u[1:], 0.0, atol=1e-14)
        errs.append(np.max(np.abs(u[0] - exact)) / exact.max())
    assert errs[0] <= 2.5e-2
    for a, b in zip(errs, errs[1:]):
        assert 3.8 <= a / b <= 4.2, errs


def test_wall_node_off_a_flat_wall_is_rejected():
    """A WALL node in a corner (two blocked axis neighbours) is not on one
    flat wall: the step fails."""
    N = 6
    fl = np.zeros(N * N, np.uint8)
    x, y, _ = inputs.grid_coords(1, N, N)
    fl[(y == 0) & (_ == 0)] = oracle.WALL
    fl[((y == 0) | (_ == 0)) & (fl == 0)] = oracle.WALL
    dom = oracle.Domain(1, N, N, periodic=1, flags=fl)
    f, _g = oracle.init(dom, np.ones(N * N), np.zeros((3, N * N)))
    with pytest.raises(RuntimeError):
        oracle.step(dom, oracle.Params(nu=0.1), f)
