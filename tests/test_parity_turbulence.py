"""GPU parity on the decaying-turbulence workload beyond one step: the whole
field at 64^3 (same spectrum cut at k = 8) over 100 steps, and the 256^3
benchmark field over 10 steps at sampled cells, each checked against the
FP64 oracle run on the cell's periodic window (the dependency cone of a
10-step pull is the cube of half-width 10 around the cell)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1807_02284_amd import inputs
from paper_1807_02284_amd.level import Level, Params
from test_parity_single import gpu_f64, odomain, oparams, rel_err

pytestmark = pytest.mark.gpu

W = oracle.weights()


def test_turbulence_64_cubed_100_steps_matches_oracle():
    """nu = 1e-5 (S = 1.99988: nearly no damping of rounding errors), adaptive
    on; both sides start from the equilibrium of the same (rho, u)."""
    n = 64
    p = Params(nu=1e-5, g_max=0.1)
    rho, u = inputs.turbulence(n, 2, 8, 0.04, seed=1807)
    lev = Level(n, n, n, p)
    lev.init_equilibrium(rho, u)
    lev.step(100)
    dom = odomain(n, n, n)
    f, _ = oracle.init(dom, rho, u)
    ref, _ = oracle.step(dom, oparams(p), f, n_steps=100)
    got, _ = gpu_f64(lev)
    assert rel_err(got, ref) <= 1e-5
    _, uo, _ = oracle.macro(dom, oparams(p), ref)
    _, ug, _ = lev.read_macro()
    ug = ug.double().cpu().numpy()
    assert np.linalg.norm(ug - uo) / np.linalg.norm(uo) <= 1e-5


HALF = 12          # window half-width: > 10 steps of pull from the wrap seam


def window(cell, n):
    """Flat indices (x fastest) of the periodic (2*HALF+1)^3 box around cell."""
    x, y, z = cell % n, (cell // n) % n, cell // (n * n)
    d = np.arange(-HALF, HALF + 1)
    xs, ys, zs = (x + d) % n, (y + d) % n, (z + d) % n
    return (xs[None, None, :] + n * (ys[None, :, None] + n * zs[:, None, None])).ravel()


def test_full_size_256_ten_steps_sampled_windows():
    """The benchmark field in the benchmark's launch configuration, 10 steps;
    cells at random and on the faces, edges and corners of the periodic box.
    The oracle runs each cell's 25^3 window with periodic wrap: the wrong
    values that the wrap brings in at the window's faces travel one cell per
    step and stay 2 cells short of the centre after 10 steps."""
    n = 256
    N = n ** 3
    steps = 10
    p = Params(nu=1e-5, g_max=0.1)
    rho, u = inputs.turbulence(n, 2, 32, 0.04, seed=1807)
    lev = Level(n, n, n, p)
    lev.init_equilibrium(rho, u)
    lev.step(steps)
    rng = np.random.default_rng(25610)
    corners = [0, n - 1, N - 1, N - n, n * n * (n - 1), n * (n - 1), n * n - 1,
               (n // 2) + n * (n // 2)]
    cells = np.unique(np.concatenate([rng.integers(0, N, 24), corners]))
    h, _ = lev.get_populations(shifted=True)
    got = h[:, torch.as_tensor(cells, device=h.device)].double().cpu().numpy() + W[:, None]
    del lev, h
    torch.cuda.empty_cache()
    m = 2 * HALF + 1
    dom = odomain(m, m, m)
    centre = HALF + m * (HALF + m * HALF)
    ref = np.empty_like(got)
    for k, c in enumerate(cells):
        idx = window(c, n)
        f, _ = oracle.init(dom, rho[idx], u[:, idx])
        fw, _ = oracle.step(dom, oparams(p), f, n_steps=steps)
        ref[:, k] = fw[:, centre]
    assert rel_err(got, ref) <= 1e-5


GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                    "turbulence64_energy.txt")


def read_golden():
    energy, spec = {}, {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("energy "):
                _, t, e = line.split()
                energy[int(t)] = float(e)
            elif line.startswith("spectrum "):
                _, k, e = line.split()
                spec[int(k)] = float(e)
    return energy, np.array([spec[k] for k in sorted(spec)])


def test_turbulence_64_cubed_1000_steps_statistics_match_the_oracle():
    """Decaying turbulence over 1000 steps at 64^3 (nu = 1e-5, adaptive on):
    beyond the first hundred steps the FP32 and FP64 trajectories part
    pointwise (a chaotic flow with almost no damping), so the comparison is
    statistical: the kinetic energy E(t) every 10 steps (within 1e-5
    relative) and the shell spectrum after 1000 steps (shells 1..16, within
    1e-4) against the oracle's (tests/golden, written by
    make_turbulence_energy.py from the oracle alone).  Measured on MI355X:
    9e-7 and 1e-5."""
    energy, spec_ref = read_golden()
    n = 64
    p = Params(nu=1e-5, g_max=0.1)
    rho, u = inputs.turbulence(n, 2, 8, 0.04, seed=1807)
    lev = Level(n, n, n, p)
    lev.init_equilibrium(rho, u)
    worst = 0.0
    for t in sorted(energy):
        if t:
            lev.step(10)
        r, ug, _ = lev.read_macro()
        e = 0.5 * float((r.double() * (ug.double() ** 2).sum(0)).sum())
        worst = max(worst, abs(e - energy[t]) / energy[t])
    print(f"E(t) largest relative deviation over 1000 steps: {worst:.3e}", flush=True)
    assert worst <= 1e-5
    U = ug.double().cpu().numpy().reshape(3, n, n, n)
    uh = np.fft.fftn(U, axes=(1, 2, 3))
    k = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    shell = np.rint(np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)).astype(int)
    e = 0.5 * np.sum(np.abs(uh) ** 2, axis=0) / float(n ** 3) ** 2
    spec = np.bincount(shell.ravel(), weights=e.ravel(), minlength=n // 2 + 1)[: n // 2 + 1]
    rel = np.abs(spec[1:17] - spec_ref[1:17]) / spec_ref[1:17]
    print("spectrum relative deviation, shells 1..16: " + " ".join(f"{x:.1e}" for x in rel), flush=True)
    assert np.max(rel) <= 1e-4
