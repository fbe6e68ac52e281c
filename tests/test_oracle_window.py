"""The premise of the sampled multi-step parity checks: k steps of the
pull-stream update at a cell depend only on the cube of half-width k around
it, so the oracle on a periodic window of half-width > k reproduces the
full-field result at the window's centre (and a window of half-width < k
does not)."""
import numpy as np

import oracle
from paper_1807_02284_amd import inputs


def periodic_window(cell, n, half):
    x, y, z = cell % n, (cell // n) % n, cell // (n * n)
    d = np.arange(-half, half + 1)
    xs, ys, zs = (x + d) % n, (y + d) % n, (z + d) % n
    return (xs[None, None, :] + n * (ys[None, :, None] + n * zs[:, None, None])).ravel()


def test_window_of_half_width_above_the_step_count_reproduces_the_full_field():
    n, steps = 20, 5
    p = oracle.Params(nu=1e-5, g_max=0.1)
    rho, u = inputs.turbulence(n, 2, 5, 0.04, seed=11)
    dom = oracle.Domain(n, n, n)
    f, _ = oracle.init(dom, rho, u)
    full, _ = oracle.step(dom, p, f, n_steps=steps)
    for half, exact in ((steps + 1, True), (steps - 2, False)):
        m = 2 * half + 1
        dw = oracle.Domain(m, m, m)
        centre = half + m * (half + m * half)
        for c in (0, n - 1, n ** 3 - 1, 4321):
            idx = periodic_window(c, n, half)
            fw, _ = oracle.init(dw, rho[idx], u[:, idx])
            r, _ = oracle.step(dw, p, fw, n_steps=steps)
            err = np.max(np.abs(r[:, centre] - full[:, c]))
            assert (err == 0.0) if exact else (err > 1e-9), (half, c, err)
