"""Adjoint of the flagged collide-stream step and of whole reference steps of
Algorithm 1 (prior-mapping, sub-steps with the fused time interpolation,
ghost remap, post-mapping), checked against central finite differences of
the FP64 oracle: the directional derivative of a linear loss of the final
states along seeded random directions of the initial states."""
import numpy as np
import pytest
import torch

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import _capi, hierarchy, inputs
from paper_1807_02284_amd.level import Level, Params
from paper_1807_02284_amd.rollout import MultiscaleRollout
from test_parity_multiscale import (Spec, build_pair, geom, gpu_g, gpu_pop, plume_specs,
                                    smooth_state, start_both)

pytestmark = pytest.mark.gpu

W = oracle.weights()


def _loss(fs, gs, Tf, Tg):
    return sum(float(np.sum(t * f)) for t, f in zip(Tf, fs)) + \
        sum(float(np.sum(t * g)) for t, g in zip(Tg, gs))


def flagged_case(kind):
    """(shape, periodic, kinds, params) of a single flagged level."""
    if kind == "plume":
        shape = (24, 12, 12)
        kinds = inputs.plume_flags(*shape, sphere_center=(9.0, 6.0, 6.0), sphere_radius=2.5,
                                   inlet_radius=4.0)
        p = Params(nu=0.02, g_max=0.5, tau_s=0.6, beta=2e-3, s_ref=0.5, u_in=(0.04, 0.0, 0.0),
                   s_in=1.0)
        return shape, 0, kinds, p
    if kind == "walls":
        # fluid up to the non-periodic y and z faces, which bounce back: the
        # adjoint's bounce-back writes cross those faces
        shape = (12, 10, 8)
        x, y, z = inputs.grid_coords(*shape)
        kinds = np.zeros(x.size, np.uint8)
        kinds[(x - 5.5) ** 2 + (y - 4.5) ** 2 + (z - 3.5) ** 2 <= 5.0] = _capi.SOLID
        kinds[(x == 0) & (y == 0)] = _capi.SOLID
        p = Params(nu=0.02, g_max=0.5, tau_s=0.6, beta=2e-3, s_ref=0.5)
        return shape, 1, kinds, p
    # an odd cell count (19 x 13 x 9 = 2223) puts Neumann copies in the last,
    # partial group of four cells of the adjoint's copy pass
    shape = (19, 13, 9) if kind == "neumann_ghost_odd" else (20, 14, 10)
    x, y, z = inputs.grid_coords(*shape)
    kinds = np.zeros(x.size, np.uint8)
    kinds[(x == 0) | (x == shape[0] - 1)] = _capi.NEUMANN
    kinds[(y == 0) | (y == shape[1] - 1)] = _capi.GHOST
    kinds[(x - 9.5) ** 2 + (y - 6.5) ** 2 + (z - 4.5) ** 2 <= 6.0] = _capi.SOLID
    p = Params(nu=0.02, g_max=0.5, tau_s=0.6)
    return shape, 4, kinds, p


@pytest.mark.parametrize("kind", ["plume", "neumann_ghost", "neumann_ghost_odd", "walls"])
def test_flagged_step_adjoint_matches_fp64_finite_differences(kind):
    shape, periodic, kinds, p = flagged_case(kind)
    n = int(np.prod(shape))
    steps = 4
    lev = Level(*shape, p, scalar=True, periodic=periodic, flags=kinds)
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.01 * rng.standard_normal(n)
    u = 0.03 * rng.standard_normal((3, n))
    s = 0.5 + 0.2 * rng.standard_normal(n)
    lev.init_equilibrium(rho, u, s)
    f0 = gpu_pop(lev)
    g0 = gpu_g(lev)
    P = lev.plane
    f_states = [torch.empty_like(lev.f) for _ in range(steps)]
    g_states = [torch.empty_like(lev.g) for _ in range(steps)]
    lev.step_store(lev.f, lev.g, f_states, g_states)
    Tf = rng.standard_normal((27, n))
    Tg = rng.standard_normal((7, n))

    def plane(x, rows):
        t = torch.zeros(rows, P, dtype=torch.float32, device="cuda")
        t[:, :n] = torch.as_tensor(x, dtype=torch.float32, device="cuda")
        return t.reshape(-1)

    lam, mu = plane(Tf, 27), plane(Tg, 7)
    lam2, mu2 = torch.zeros_like(lam), torch.zeros_like(mu)
    inputs_f = [lev.f] + f_states[:-1]
    inputs_g = [lev.g] + g_states[:-1]
    for k in reversed(range(steps)):
        lev.adjoint_step(inputs_f[k], inputs_g[k], lam, mu, lam2, mu2, None)
        lam, lam2 = lam2, lam
        mu, mu2 = mu2, mu
    gf = lam.reshape(27, P)[:, :n].double().cpu().numpy()
    gg = mu.reshape(7, P)[:, :n].double().cpu().numpy()

    op = oracle.Params(nu=p.nu, g_max=p.g_max, tau_s=p.tau_s, beta=p.beta, s_ref=p.s_ref)
    dom = oracle.Domain(*shape, periodic=periodic, flags=kinds, u_in=p.u_in, s_in=p.s_in)

    def L(df, dg):
        f, g = oracle.step(dom, op, f0 + df, g0 + dg, n_steps=steps)
        return _loss([f], [g], [Tf], [Tg])

    for seed in (11, 12):
        r = np.random.default_rng(seed)
        df = 1e-4 * r.standard_normal((27, n))
        dg = 1e-4 * r.standard_normal((7, n))
        eps = 1.0
        fd = (L(eps * df, eps * dg) - L(-eps * df, -eps * dg)) / (2 * eps)
        ad = float(np.sum(gf * df) + np.sum(gg * dg))
        assert ad == pytest.approx(fd, rel=1e-3), (seed, ad, fd)


@pytest.mark.parametrize("kind", ["plume", "neumann_ghost", "neumann_ghost_odd", "walls"])
def test_flagged_step_adjoint_writes_every_element(kind):
    """The flagged adjoint writes each element of its outputs itself (the
    value, or zero where no fluid cell pulls it) and clears the plane
    padding: outputs that start as NaN end bit-equal to outputs that start
    as zero."""
    shape, periodic, kinds, p = flagged_case(kind)
    n = int(np.prod(shape))
    lev = Level(*shape, p, scalar=True, periodic=periodic, flags=kinds)
    rng = np.random.default_rng(7)
    lev.init_equilibrium(1.0 + 0.01 * rng.standard_normal(n), 0.03 * rng.standard_normal((3, n)),
                         0.5 + 0.2 * rng.standard_normal(n))
    # the flag preparation marks the non-fluid cells with a fluid cell among
    # their 26 neighbours (periodic wrap on every axis)
    k3 = kinds.reshape(shape[::-1])
    near = np.zeros_like(k3, dtype=bool)
    for d in np.ndindex(3, 3, 3):
        near |= np.roll(k3 == _capi.FLUID, tuple(np.array(d) - 1), axis=(0, 1, 2))
    got = lev.flags[:n].cpu().numpy().reshape(shape[::-1])
    np.testing.assert_array_equal((got & _capi.NEAR_FLUID) != 0, near & (k3 != _capi.FLUID))
    assert np.array_equal(got & 7, k3)
    P = lev.plane
    lam = torch.zeros(27, P, device="cuda")
    mu = torch.zeros(7, P, device="cuda")
    lam[:, :n] = torch.as_tensor(rng.standard_normal((27, n)), dtype=torch.float32, device="cuda")
    mu[:, :n] = torch.as_tensor(rng.standard_normal((7, n)), dtype=torch.float32, device="cuda")
    lam, mu = lam.reshape(-1), mu.reshape(-1)
    outs = []
    for fill in (0.0, float("nan")):
        lam0 = torch.full_like(lam, fill)
        mu0 = torch.full_like(mu, fill)
        lev.adjoint_step(lev.f, lev.g, lam, mu, lam0, mu0, None)
        torch.cuda.synchronize()
        outs.append((lam0.cpu().numpy(), mu0.cpu().numpy()))
    (a, b), (c, d) = outs
    assert np.all(np.isfinite(c)) and np.all(np.isfinite(d))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
    assert np.array_equal(b.view(np.uint32), d.view(np.uint32))
    assert not a.reshape(27, P)[:, n:].any() and not b.reshape(7, P)[:, n:].any()
    # solid cells that no fluid cell bounces into keep a zero adjoint
    deep = (kinds == _capi.SOLID)
    for axis in range(3):
        k3 = (kinds == _capi.SOLID).reshape(shape[::-1])
        deep &= np.roll(k3, 1, axis).reshape(-1) & np.roll(k3, -1, axis).reshape(-1)
    if deep.any():
        assert not a.reshape(27, P)[:, :n][:, deep].any()


def _exchange_adjoint_gpu(lev_src, lev_dst, cells, w, fA, fB, gA, gB, lam_d, mu_d, gather=False):
    import ctypes as C
    cells_t = torch.as_tensor(np.asarray(cells, np.int32), device="cuda")
    lev_src._sync_struct()
    lev_dst._sync_struct()
    lam_a, lam_b = torch.zeros_like(fA), torch.zeros_like(fA)
    mu_a, mu_b = torch.zeros_like(gA), torch.zeros_like(gA)
    ws, nbytes = None, 0
    if gather:
        lib = _capi.load()
        nbytes = lib.cslbm_exchange_adjoint_bytes(C.byref(lev_src.c), C.byref(lev_dst.c),
                                                  int(cells_t.numel()))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    _capi.call("cslbm_exchange_adjoint", C.byref(lev_src.c), fA.data_ptr(), fB.data_ptr(),
               gA.data_ptr(), gB.data_ptr(), float(w), C.byref(lev_dst.c), lam_d.data_ptr(),
               mu_d.data_ptr(), lam_a.data_ptr(), lam_b.data_ptr(), mu_a.data_ptr(),
               mu_b.data_ptr(), cells_t.data_ptr(), int(cells_t.numel()),
               None if ws is None else ws.data_ptr(), int(nbytes),
               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return lam_a, lam_b, mu_a, mu_b


@pytest.mark.parametrize("gather", [False, True])
@pytest.mark.parametrize("case", ["prior_blend", "post", "post_node"])
def test_exchange_adjoint_matches_fp64_finite_differences(case, gather):
    n = 20
    nu0 = 2e-3
    coarse = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    if case == "post_node":
        fshape = (22, 20, 18)
        fine = Spec(fshape, (4.5, 5.0, 3.5), 0.5, nu0, hierarchy.shell_flags(*fshape))
    else:
        fshape = (19, 19, 17)
        fine = Spec(fshape, (5.3, 5.4, 5.6), 1 / 1.5, nu0, hierarchy.shell_flags(*fshape))
    levC, _ = start_both(coarse, 6)
    levC2, _ = start_both(coarse, 8)
    levF, _ = start_both(fine, 7)
    if case == "prior_blend":
        src, dst, spec_s, spec_d, w = levC, levF, coarse, fine, 0.37
        cells = np.flatnonzero(fine.kinds == _capi.GHOST)
        fA, fB, gA, gB = levC.f, levC2.f, levC.g, levC2.g
    else:
        src, dst, spec_s, spec_d, w = levF, levC, fine, coarse, 0.0
        cells = hierarchy.post_cells(coarse.kinds, coarse.shape, coarse.origin, 1.0, fine.kinds,
                                     fine.shape, fine.origin, fine.dx)
        fA, fB, gA, gB = levF.f, levF.f, levF.g, levF.g
    assert cells.size > 100
    rng = np.random.default_rng(3)
    Tf = rng.standard_normal((27, dst.n))
    Tg = rng.standard_normal((7, dst.n))

    def plane(x, rows, lev):
        t = torch.zeros(rows, lev.plane, dtype=torch.float32, device="cuda")
        t[:, : lev.n] = torch.as_tensor(x, dtype=torch.float32, device="cuda")
        return t.reshape(-1)

    lam_d, mu_d = plane(Tf, 27, dst), plane(Tg, 7, dst)
    la, lb, ma, mb = _exchange_adjoint_gpu(src, dst, cells, w, fA, fB, gA, gB, lam_d, mu_d, gather)
    # the targets' adjoints are cleared, the others kept
    ld = lam_d.reshape(27, dst.plane)[:, : dst.n].cpu().numpy()
    assert np.all(ld[:, cells] == 0.0)
    keep = np.setdiff1d(np.arange(dst.n), cells)
    assert np.array_equal(ld[:, keep], Tf[:, keep].astype(np.float32))

    def dense(t, rows, lev):
        return t.reshape(rows, lev.plane)[:, : lev.n].double().cpu().numpy()

    A, B = dense(fA, 27, src) + W[:, None], dense(fB, 27, src) + W[:, None]
    GA, GB = dense(gA, 7, src), dense(gB, 7, src)
    base_f = dense(dst.f, 27, dst) + W[:, None]
    base_g = dense(dst.g, 7, dst)

    def L(dA, dB, dgA, dgB):
        fo, go = base_f.copy(), base_g.copy()
        oracle.exchange(geom(spec_s), A + dA, B + dB, w, geom(spec_d), cells.astype(np.int64), fo,
                        GA + dgA, GB + dgB, go)
        return float(np.sum(Tf * fo) + np.sum(Tg * go))

    gla, glb = dense(la, 27, src), dense(lb, 27, src)
    gma, gmb = dense(ma, 7, src), dense(mb, 7, src)
    for seed in (41, 42):
        r = np.random.default_rng(seed)
        dA, dB = 1e-4 * r.standard_normal(A.shape), 1e-4 * r.standard_normal(A.shape)
        dgA, dgB = 1e-4 * r.standard_normal(GA.shape), 1e-4 * r.standard_normal(GA.shape)
        if case != "prior_blend":         # one source state read twice
            dB, dgB = dA, dgA
        fd = (L(dA, dB, dgA, dgB) - L(-dA, -dB, -dgA, -dgB)) / 2.0
        ad = float(np.sum(gla * dA) + np.sum(glb * dB) + np.sum(gma * dgA) + np.sum(gmb * dgB))
        assert ad == pytest.approx(fd, rel=1e-4), (seed, ad, fd)


@pytest.mark.parametrize("case", ["prior_blend", "post", "post_node", "wrapping"])
def test_exchange_adjoint_gather_equals_atomic_scatter(case):
    """The gather form and the atomic scatter sum the same contributions
    (different order); "wrapping" puts targets whose stencil wraps around a
    periodic source box next to interior ones."""
    n = 20
    nu0 = 2e-3
    coarse = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    if case == "post_node":
        fshape = (22, 20, 18)
        fine = Spec(fshape, (4.5, 5.0, 3.5), 0.5, nu0, hierarchy.shell_flags(*fshape))
    elif case == "wrapping":
        fshape = (12, 10, 9)
        fine = Spec(fshape, (14.2, 3.3, 5.1), 1 / 1.5, nu0, hierarchy.shell_flags(*fshape))
    else:
        fshape = (19, 19, 17)
        fine = Spec(fshape, (5.3, 5.4, 5.6), 1 / 1.5, nu0, hierarchy.shell_flags(*fshape))
    levC, _ = start_both(coarse, 6)
    levC2, _ = start_both(coarse, 8)
    levF, _ = start_both(fine, 7)
    if case in ("prior_blend", "wrapping"):
        src, dst, w = levC, levF, 0.37
        cells = np.arange(fine.n) if case == "wrapping" else np.flatnonzero(fine.kinds == _capi.GHOST)
        fA, fB, gA, gB = levC.f, levC2.f, levC.g, levC2.g
    else:
        src, dst, w = levF, levC, 0.0
        cells = hierarchy.post_cells(coarse.kinds, coarse.shape, coarse.origin, 1.0, fine.kinds,
                                     fine.shape, fine.origin, fine.dx)
        fA, fB, gA, gB = levF.f, levF.f, levF.g, levF.g
    rng = np.random.default_rng(4)
    out = []
    for gather in (False, True):
        lam_d = torch.zeros(27, dst.plane, device="cuda")
        lam_d[:, : dst.n] = torch.as_tensor(rng.standard_normal((27, dst.n)) if not out else Tf,
                                            dtype=torch.float32, device="cuda")
        if not out:
            Tf = lam_d[:, : dst.n].cpu().numpy().astype(np.float64)
        mu_d = torch.zeros(7, dst.plane, device="cuda")
        mu_d[:, : dst.n] = 0.5
        res = _exchange_adjoint_gpu(src, dst, cells, w, fA, fB, gA, gB, lam_d.reshape(-1),
                                    mu_d.reshape(-1), gather)
        out.append([r.cpu().numpy() for r in res])
    for a, b in zip(*out):
        scale = max(np.max(np.abs(a)), 1e-30)
        assert np.max(np.abs(a - b)) <= 1e-5 * scale


def chain_specs(nu0=2e-3, adaptive=True):
    n = 24
    s0 = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    sh1 = (19, 19, 17)
    s1 = Spec(sh1, (5.3, 5.4, 5.6), 1 / 1.5, nu0, hierarchy.shell_flags(*sh1), parent=0)
    sh2 = (14, 13, 12)
    s2 = Spec(sh2, (8.1, 8.3, 8.2), 0.5, nu0, hierarchy.shell_flags(*sh2), parent=1)
    for sp in (s0, s1, s2):
        sp.adaptive = adaptive
    return [s0, s1, s2]


# The adaptive factor phi(G), G = sqrt(2 S:S), is a norm of the
# non-equilibrium stress.  With S close to 2 (nu0 = 2e-3: S = 1.976 on the
# reference scale) the stress left by the previous collision, -(1 - S)
# times the old one, nearly cancels the stress the pull creates, so at every
# other step G is small at most cells and its derivative (the stress
# direction) is fixed by digits that differ between the FP32 and the FP64
# trajectory: the FP32 adjoint and the FP64 finite difference then differ
# by about 1e-3 after a few steps for a reason that is not an error in
# either.  The schedule is therefore checked with the adaptive factor off
# (a smooth map: tight tolerance) and, with it on, at nu0 = 2e-2 (S = 1.79),
# where the stress does not cancel.
@pytest.mark.parametrize("n_scales,n_ref,every,nu0,adaptive,tol",
                         [(2, 3, 2, 2e-3, False, 2e-5), (3, 3, 2, 2e-3, False, 2e-5),
                          (3, 2, 1, 2e-2, True, 2e-4)])
def test_multiscale_adjoint_matches_fp64_finite_differences(n_scales, n_ref, every, nu0, adaptive,
                                                            tol):
    specs = chain_specs(nu0, adaptive)[:n_scales]
    H, levs, oscs = build_pair(specs, 20)
    f0 = [gpu_pop(lev) for lev in levs]
    g0 = [gpu_g(lev) for lev in levs]
    ro = MultiscaleRollout(H, every=every)
    ro.forward(n_ref)
    rng = np.random.default_rng(7)
    Tf = [rng.standard_normal((27, lev.n)) for lev in levs]
    Tg = [rng.standard_normal((7, lev.n)) for lev in levs]
    lf, lg = ro.backward([torch.as_tensor(t, dtype=torch.float32, device="cuda") for t in Tf],
                         [torch.as_tensor(t, dtype=torch.float32, device="cuda") for t in Tg])
    gf = [x.double().cpu().numpy() for x in lf]
    gg = [x.double().cpu().numpy() for x in lg]
    # the rollout leaves the scales in their final forward state
    fin = [gpu_pop(lev) for lev in levs]

    def run_oracle(df, dg):
        sc = [sp.oscale() for sp in specs]
        for s, a, b, da, db in zip(sc, f0, g0, df, dg):
            s.f, s.g = a + da, b + db
        ml.prepare(sc)
        ml.multiscale_step(sc, n_ref)
        return sc

    base = run_oracle([0 * f for f in f0], [0 * g for g in g0])
    for lev, s, x in zip(levs, base, fin):
        assert np.max(np.abs(x - s.f) / np.maximum(np.abs(s.f), W[:, None])) <= 1e-5

    # Directions of amplitude 1e-7: where G is small it bends sharply, and
    # larger steps leave an O(step) error in the central difference of the
    # adaptive factor (one 24^3 step: 3e-3 relative at 1e-4, 2e-6 at 1e-7).
    for seed in (31, 32):
        r = np.random.default_rng(seed)
        df = [1e-7 * r.standard_normal(f.shape) for f in f0]
        dg = [1e-7 * r.standard_normal(g.shape) for g in g0]
        sp = run_oracle(df, dg)
        sm = run_oracle([-d for d in df], [-d for d in dg])
        fd = (_loss([s.f for s in sp], [s.g for s in sp], Tf, Tg) -
              _loss([s.f for s in sm], [s.g for s in sm], Tf, Tg)) / 2.0
        ad = sum(float(np.sum(a * d)) for a, d in zip(gf, df)) + \
            sum(float(np.sum(a * d)) for a, d in zip(gg, dg))
        assert ad == pytest.approx(fd, rel=tol), (seed, ad, fd)


def test_reduced_plume_multiscale_adjoint_matches_fp64_finite_differences():
    """The three-scale plume scene at 96x48x48 (walls, inlet, outflow, a
    sphere on every scale, spacing ratios 1.5 and 2), two reference steps,
    adaptive factor off."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    levs, oscs = [], []
    for sp in specs:
        sp.adaptive = False           # a smooth map for the finite difference (see above)
        rho, u, s = smooth_state(sp, 40)
        u[0] += 0.04
        lev = sp.level(True)
        lev.init_equilibrium(rho, u, s)
        levs.append(lev)
    # post-mapping lists in tiles (each run mapped through LDS)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs],
                            tile_min_fill=0)
    assert H.c_scales[2].n_post_tiles[1] > 0 and H.c_scales[1].n_post_tiles[0] > 0
    f0 = [gpu_pop(lev) for lev in levs]
    g0 = [gpu_g(lev) for lev in levs]
    n_ref = 2
    ro = MultiscaleRollout(H, every=1)
    ro.forward(n_ref)
    rng = np.random.default_rng(9)
    Tf = [rng.standard_normal((27, lev.n)) for lev in levs]
    Tg = [rng.standard_normal((7, lev.n)) for lev in levs]
    lf, lg = ro.backward([torch.as_tensor(t, dtype=torch.float32, device="cuda") for t in Tf],
                         [torch.as_tensor(t, dtype=torch.float32, device="cuda") for t in Tg])
    gf = [x.double().cpu().numpy() for x in lf]
    gg = [x.double().cpu().numpy() for x in lg]

    def run_oracle(df, dg):
        sc = [sp.oscale() for sp in specs]
        for s_, a, b, da, db in zip(sc, f0, g0, df, dg):
            s_.f, s_.g = a + da, b + db
        ml.prepare(sc)
        ml.multiscale_step(sc, n_ref)
        return sc

    r = np.random.default_rng(51)
    df = [1e-7 * r.standard_normal(f.shape) for f in f0]
    dg = [1e-7 * r.standard_normal(g.shape) for g in g0]
    sp_ = run_oracle(df, dg)
    sm_ = run_oracle([-d for d in df], [-d for d in dg])
    fd = (_loss([s_.f for s_ in sp_], [s_.g for s_ in sp_], Tf, Tg) -
          _loss([s_.f for s_ in sm_], [s_.g for s_ in sm_], Tf, Tg)) / 2.0
    ad = sum(float(np.sum(a * d)) for a, d in zip(gf, df)) + \
        sum(float(np.sum(a * d)) for a, d in zip(gg, dg))
    assert ad == pytest.approx(fd, rel=2e-5), (ad, fd)


@pytest.mark.parametrize("plates", ["never", "always"])
def test_tiled_post_mapping_adjoint_gives_bitwise_the_gathered_adjoint(plates):
    """With the post-mapping lists in tile runs (plane tiles, or tiles lying
    in the lists' plates), each run's interpolation and
    map adjoint run in one workgroup through LDS: the columns, index map and
    flags are those of the per-target passes, so one multi-scale adjoint step
    of the reduced plume is bitwise that of the untiled lists."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    out = []
    for tiles in (True, False):
        levs = []
        for sp in specs:
            rho, u, s = smooth_state(sp, 40)
            u[0] += 0.04
            lev = sp.level(True)
            lev.init_equilibrium(rho, u, s)
            levs.append(lev)
        H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs],
                                tile_posts=tiles, tile_min_fill=0, tile_plates=plates)
        assert (H.c_scales[2].n_post_tiles[1] > 0) == tiles
        assert (H.c_scales[1].n_post_tiles[0] > 0) == tiles
        H.step(2)
        f_in = [lev.f.clone() for lev in levs]
        g_in = [lev.g.clone() for lev in levs]
        gen = torch.Generator(device="cuda").manual_seed(5)
        lam = [torch.randn(27 * lev.plane, device="cuda", generator=gen) for lev in levs]
        mu = [torch.randn(7 * lev.plane, device="cuda", generator=gen) for lev in levs]
        ws = torch.empty(H.adjoint_workspace_bytes(), dtype=torch.uint8, device="cuda")
        H.adjoint_step(f_in, g_in, lam, mu, ws)
        torch.cuda.synchronize()
        out.append([x.cpu().numpy() for x in lam + mu])
        assert all(np.all(np.isfinite(x)) for x in out[-1])
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_staged_shell_interpolation_gives_bitwise_the_unstaged_adjoint():
    """The interpolation pass of the ghost-shell adjoints reads the x-face
    entries from the staged copies of the parent's columns, as the forward
    step does: one multi-scale adjoint step of the reduced plume is bitwise
    that of the hierarchy without staging, with a stage per scale (the
    recompute's copies are read) and with one stage shared by both finer
    scales (each scale's copy is made again before its adjoints)."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    out = []
    for mode in ("private", "shared", "unstaged"):
        staged = mode != "unstaged"
        levs = []
        for sp in specs:
            rho, u, s = smooth_state(sp, 40)
            u[0] += 0.04
            lev = sp.level(True)
            lev.init_equilibrium(rho, u, s)
            levs.append(lev)
        H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs],
                                stage_xfaces=staged)
        for i in (1, 2):
            sc = H.c_scales[i]
            assert bool(sc.stage) == staged and (sc.n_ghost_xlo > 0) == staged
        if mode == "shared":
            shared = torch.empty(max(H.c_scales[i].stage_bytes for i in (1, 2)), dtype=torch.uint8,
                                 device="cuda")
            for i in (1, 2):
                H.c_scales[i].stage = shared.data_ptr()
        H.step(2)
        f_in = [lev.f.clone() for lev in levs]
        g_in = [lev.g.clone() for lev in levs]
        gen = torch.Generator(device="cuda").manual_seed(7)
        lam = [torch.randn(27 * lev.plane, device="cuda", generator=gen) for lev in levs]
        mu = [torch.randn(7 * lev.plane, device="cuda", generator=gen) for lev in levs]
        ws = torch.empty(H.adjoint_workspace_bytes(), dtype=torch.uint8, device="cuda")
        H.adjoint_step(f_in, g_in, lam, mu, ws)
        torch.cuda.synchronize()
        out.append([x.cpu().numpy() for x in lam + mu])
        assert all(np.all(np.isfinite(x)) for x in out[-1])
    for other in out[:2]:
        for a, b in zip(other, out[2]):
            np.testing.assert_array_equal(a, b)


def test_shell_patch_recompute_gives_bitwise_the_gathered_adjoint():
    """The forward recompute of the multi-scale adjoint maps the ghost
    shells in patch runs through LDS as the forward step does: one
    multi-scale adjoint step of the reduced plume is bitwise that of the
    hierarchy whose shells are gathered directly (the adjoint passes sum
    each source cell's targets in the order of their positions, whatever
    the order of the list)."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    out = []
    for tiles in (True, False):
        levs = []
        for sp in specs:
            rho, u, s = smooth_state(sp, 40)
            u[0] += 0.04
            lev = sp.level(True)
            lev.init_equilibrium(rho, u, s)
            levs.append(lev)
        H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs],
                                tile_shells=tiles)
        assert all((H.c_scales[i].n_ghost_tiles > 0) == tiles for i in (1, 2))
        H.step(2)
        f_in = [lev.f.clone() for lev in levs]
        g_in = [lev.g.clone() for lev in levs]
        gen = torch.Generator(device="cuda").manual_seed(9)
        lam = [torch.randn(27 * lev.plane, device="cuda", generator=gen) for lev in levs]
        mu = [torch.randn(7 * lev.plane, device="cuda", generator=gen) for lev in levs]
        ws = torch.empty(H.adjoint_workspace_bytes(), dtype=torch.uint8, device="cuda")
        H.adjoint_step(f_in, g_in, lam, mu, ws)
        torch.cuda.synchronize()
        out.append([x.cpu().numpy() for x in lam + mu])
        assert all(np.all(np.isfinite(x)) for x in out[-1])
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_multiscale_adjoint_scope_is_checked():
    specs = chain_specs()
    specs[2].parent = 0                       # not a chain
    H, _, _ = build_pair(specs, 21)
    with pytest.raises(_capi.CslbmError):
        H.adjoint_workspace_bytes()


def test_multiscale_adjoint_over_the_fp64_trajectory_with_the_adaptive_factor():
    """Three scales at nu0 = 2e-3 (S = 1.976 on the reference scale) with the
    adaptive factor on, four reference steps.  The adjoint of each reference
    step is evaluated at the oracle's FP64 state at its start (rounded to
    FP32), so the chained adjoint is compared with central differences of
    the FP64 oracle without the FP32 trajectory's drift in the direction of
    a small non-equilibrium stress (which sets the adaptive factor's
    derivative)."""
    specs = chain_specs(2e-3, True)
    H, levs, oscs = build_pair(specs, 20)
    n_ref = 4
    f0 = [gpu_pop(lev) for lev in levs]
    g0 = [gpu_g(lev) for lev in levs]

    def oracle_from(df, dg):
        sc = [sp.oscale() for sp in specs]
        for s, a, b, da, db in zip(sc, f0, g0, df, dg):
            s.f, s.g = a + da, b + db
        ml.prepare(sc)
        return sc

    sc = oracle_from([0 * f for f in f0], [0 * g for g in g0])
    traj = [([s.f.copy() for s in sc], [s.g.copy() for s in sc])]
    for _ in range(n_ref):
        ml.multiscale_step(sc, 1)
        traj.append(([s.f.copy() for s in sc], [s.g.copy() for s in sc]))

    def planes(lev, x, rows):
        t = torch.zeros(rows, lev.plane, dtype=torch.float32, device="cuda")
        t[:, : lev.n] = torch.as_tensor(np.asarray(x).reshape(rows, lev.n), dtype=torch.float32,
                                        device="cuda")
        return t.reshape(-1)

    rng = np.random.default_rng(7)
    Tf = [rng.standard_normal((27, lev.n)) for lev in levs]
    Tg = [rng.standard_normal((7, lev.n)) for lev in levs]
    lam = [planes(lev, t, 27) for lev, t in zip(levs, Tf)]
    mu = [planes(lev, t, 7) for lev, t in zip(levs, Tg)]
    ws = torch.empty(H.adjoint_workspace_bytes(), dtype=torch.uint8, device="cuda")
    for n in reversed(range(n_ref)):
        fs, gs = traj[n]
        f_in = [planes(lev, f - W[:, None], 27) for lev, f in zip(levs, fs)]
        g_in = [planes(lev, g, 7) for lev, g in zip(levs, gs)]
        H.adjoint_step(f_in, g_in, lam, mu, ws)
    torch.cuda.synchronize()
    gf = [l.reshape(27, lev.plane)[:, : lev.n].double().cpu().numpy() for l, lev in zip(lam, levs)]
    gg = [m.reshape(7, lev.plane)[:, : lev.n].double().cpu().numpy() for m, lev in zip(mu, levs)]
    for seed in (41, 42, 43):
        r = np.random.default_rng(seed)
        df = [1e-7 * r.standard_normal(f.shape) for f in f0]
        dg = [1e-7 * r.standard_normal(g.shape) for g in g0]
        sp = oracle_from(df, dg)
        ml.multiscale_step(sp, n_ref)
        sm = oracle_from([-d for d in df], [-d for d in dg])
        ml.multiscale_step(sm, n_ref)
        fd = (_loss([s.f for s in sp], [s.g for s in sp], Tf, Tg) -
              _loss([s.f for s in sm], [s.g for s in sm], Tf, Tg)) / 2.0
        ad = sum(float(np.sum(a * d)) for a, d in zip(gf, df)) + \
            sum(float(np.sum(a * d)) for a, d in zip(gg, dg))
        print(f"direction {seed}: adjoint {ad:.9e}, central difference {fd:.9e}", flush=True)
        assert ad == pytest.approx(fd, rel=2e-4), (seed, ad, fd)
