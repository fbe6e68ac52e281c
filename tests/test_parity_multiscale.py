"""GPU parity of the cross-scale exchange, temporal interpolation and the
Algorithm-1 driver against the FP64 oracle (same seeded inputs, same scale
geometry)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import _capi, hierarchy, inputs
from paper_1807_02284_amd.level import F16S, F32, Level, Params

pytestmark = pytest.mark.gpu

W = oracle.weights()


def rel_err(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), W[:, None]))


def gpu_pop(lev: Level, buf=None):
    """Physical populations (float64 [27][N]) of a level's state or of any
    [27][plane] buffer of it."""
    t = lev.f if buf is None else buf
    h = t.reshape(27, lev.plane)[:, : lev.n].double().cpu().numpy()
    return h + W[:, None]


def gpu_g(lev: Level, buf=None):
    t = lev.g if buf is None else buf
    return t.reshape(7, lev.plane)[:, : lev.n].double().cpu().numpy()


class Spec:
    """One scale: box size, origin, spacing, kinds; builds both sides."""

    def __init__(self, shape, origin, dx, nu0, kinds, periodic=0, parent=-1, tau_s0=0.55,
                 u_in=(0.0, 0.0, 0.0), s_in=0.0):
        self.shape, self.origin, self.dx = shape, origin, dx
        self.alpha = 1.0 / dx
        self.nu = nu0 * self.alpha
        self.tau_s = 0.5 + self.alpha * (tau_s0 - 0.5)
        self.kinds, self.periodic, self.parent = kinds, periodic, parent
        self.u_in, self.s_in = u_in, s_in
        self.adaptive = True

    @property
    def n(self):
        return int(np.prod(self.shape))

    def params(self):
        return Params(nu=self.nu, g_max=0.05, tau_s=self.tau_s, u_in=self.u_in, s_in=self.s_in,
                      adaptive=self.adaptive)

    def level(self, scalar):
        flags = None if (self.periodic == 7 and np.all(self.kinds == 0)) else self.kinds
        return Level(*self.shape, self.params(), scalar=scalar, periodic=self.periodic, flags=flags,
                     origin=self.origin, dx=self.dx)

    def oscale(self):
        p = self.params()
        return ml.OScale(*self.shape, self.dx, self.origin,
                         oracle.Params(nu=p.nu, g_max=p.g_max, tau_s=p.tau_s, adaptive=p.adaptive),
                         self.kinds,
                         periodic=self.periodic, parent=self.parent, u_in=self.u_in, s_in=self.s_in)

    def positions(self):
        x, y, z = inputs.grid_coords(*self.shape)
        return (self.origin[0] + x * self.dx, self.origin[1] + y * self.dx,
                self.origin[2] + z * self.dx)


def smooth_state(spec: Spec, seed):
    """(rho, u, s) sampled at the scale's physical points from one seeded
    smooth field defined on the whole domain."""
    px, py, pz = spec.positions()
    rng = np.random.default_rng(seed)
    u = np.zeros((3, px.size))
    for a in range(3):
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            u[a] += 0.015 * np.cos(2 * np.pi * (k[0] * px + k[1] * py + k[2] * pz) / 24.0 + ph)
    rho = 1.0 + 0.005 * np.sin(2 * np.pi * (px + 2 * py) / 24.0)
    s = 0.5 + 0.3 * np.cos(2 * np.pi * (px - pz) / 24.0)
    return rho, u, s


def start_both(spec: Spec, seed, scalar=True):
    rho, u, s = smooth_state(spec, seed)
    lev = spec.level(scalar)
    lev.init_equilibrium(rho, u, s if scalar else None)
    osc = spec.oscale()
    osc.f, osc.g = oracle.init(osc.domain(), rho, u, s=s if scalar else None)
    return lev, osc


def geom(spec: Spec, scalar=True):
    return dict(nx=spec.shape[0], ny=spec.shape[1], nz=spec.shape[2], periodic=spec.periodic,
                origin=spec.origin, dx=spec.dx, nu=spec.nu, tau_s=spec.tau_s if scalar else 0.0)


@pytest.mark.parametrize("dst_dx,w", [(1 / 1.5, 0.37), (0.5, 0.0), (1 / 1.25, 1.0)])
def test_exchange_coarse_to_fine_matches_oracle(dst_dx, w):
    n = 24
    src = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, 2e-3, np.zeros(n ** 3, np.uint8), periodic=7)
    dshape = (15, 13, 12)
    dst = Spec(dshape, (3.3, 2.6, 17.1), dst_dx, 2e-3, hierarchy.shell_flags(*dshape))
    levA, oA = start_both(src, 1)
    levB, oB = start_both(src, 2)
    levD, oD = start_both(dst, 3)
    cells = np.arange(dst.n, dtype=np.int32)
    cells_t = torch.as_tensor(cells, device="cuda")
    levA._sync_struct(); levB._sync_struct(); levD._sync_struct()
    import ctypes as C
    _capi.call("cslbm_exchange", C.byref(levA.c), levA.f.data_ptr(), levB.f.data_ptr(),
               levA.g.data_ptr(), levB.g.data_ptr(), float(w), C.byref(levD.c), levD.f.data_ptr(),
               levD.g.data_ptr(), cells_t.data_ptr(), cells.size,
               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    fo, go = oD.f.copy(), oD.g.copy()
    oracle.exchange(geom(src), oA.f, oB.f, w, geom(dst), cells.astype(np.int64), fo, oA.g, oB.g, go)
    assert rel_err(gpu_pop(levD), fo) <= 1e-6
    assert np.max(np.abs(gpu_g(levD) - go)) <= 2e-7


def test_exchange_fine_to_coarse_matches_oracle():
    n = 24
    coarse = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, 2e-3, np.zeros(n ** 3, np.uint8), periodic=7)
    fshape = (20, 18, 16)
    fine = Spec(fshape, (4.2, 5.1, 3.7), 1 / 1.5, 2e-3, hierarchy.shell_flags(*fshape))
    levC, oC = start_both(coarse, 4)
    levF, oF = start_both(fine, 5)
    cells = hierarchy.post_cells(coarse.kinds, coarse.shape, coarse.origin, 1.0, fine.kinds,
                                 fine.shape, fine.origin, fine.dx)
    assert cells.size > 100
    cells_t = torch.as_tensor(cells, device="cuda")
    import ctypes as C
    levC._sync_struct(); levF._sync_struct()
    _capi.call("cslbm_exchange", C.byref(levF.c), levF.f.data_ptr(), None, levF.g.data_ptr(), None,
               0.0, C.byref(levC.c), levC.f.data_ptr(), levC.g.data_ptr(), cells_t.data_ptr(),
               cells.size, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    fo, go = oC.f.copy(), oC.g.copy()
    oracle.exchange(geom(fine), oF.f, oF.f, 0.0, geom(coarse), cells.astype(np.int64), fo, oF.g,
                    oF.g, go)
    assert rel_err(gpu_pop(levC), fo) <= 1e-6
    assert np.max(np.abs(gpu_g(levC) - go)) <= 2e-7


def test_time_interp_matches_oracle():
    spec = Spec((30, 7, 5), (0.0, 0.0, 0.0), 1.0, 1e-3, np.zeros(1050, np.uint8), periodic=7)
    levs, ors = zip(*[start_both(spec, 10 + k) for k in range(3)])
    out = Level(*spec.shape, spec.params(), scalar=True)
    import ctypes as C
    t = (C.c_double * 3)(0.0, 2.0 / 3.0, 4.0 / 3.0)
    out._sync_struct()
    _capi.call("cslbm_time_interp", C.byref(out.c), levs[0].f.data_ptr(), levs[1].f.data_ptr(),
               levs[2].f.data_ptr(), levs[0].g.data_ptr(), levs[1].g.data_ptr(),
               levs[2].g.data_ptr(), t, 1.0, out.f.data_ptr(), out.g.data_ptr(),
               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = oracle.time_interp(ors[0].f, ors[1].f, ors[2].f, tuple(t), 1.0).reshape(27, -1)
    gref = oracle.time_interp(ors[0].g, ors[1].g, ors[2].g, tuple(t), 1.0).reshape(7, -1)
    assert rel_err(gpu_pop(out), ref) <= 1e-6
    assert np.max(np.abs(gpu_g(out) - gref)) <= 1e-6


def build_pair(specs, seed, scalar=True):
    levs, oscs = [], []
    for i, sp in enumerate(specs):
        lev, osc = start_both(sp, seed, scalar)      # one physical field on every scale
        levs.append(lev)
        oscs.append(osc)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs])
    ml.prepare(oscs)
    for i in range(1, len(specs)):
        np.testing.assert_array_equal(np.sort(H.post_full[(i, 0)].astype(np.int64)), oscs[i].post[0])
    return H, levs, oscs


def test_three_scale_reference_steps_match_oracle():
    n = 24
    nu0 = 2e-3
    s0 = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    sh1 = (19, 19, 17)
    s1 = Spec(sh1, (5.3, 5.4, 5.6), 1 / 1.5, nu0, hierarchy.shell_flags(*sh1), parent=0)
    sh2 = (14, 13, 12)
    s2 = Spec(sh2, (8.1, 8.3, 8.2), 0.5, nu0, hierarchy.shell_flags(*sh2), parent=1)
    H, levs, oscs = build_pair([s0, s1, s2], 20)
    H.step(3)
    ml.multiscale_step(oscs, 3)
    torch.cuda.synchronize()
    for lev, osc in zip(levs, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5


def test_sibling_scales_of_the_reference_match_oracle():
    """Two finer scales that are both children of the reference scale, the
    second overlapping the first: scale 2's prior-mappings read reference
    cells that scale 1 has post-mapped, and scale 2 also post-maps into
    scale 1.  The library runs post-mappings on a second stream; the
    reference-scale reads of scale 2 must wait for scale 1's post into the
    reference, as Algorithm 1 orders them."""
    n = 24
    nu0 = 2e-3
    s0 = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    sh1 = (13, 12, 12)
    s1 = Spec(sh1, (2.3, 5.4, 5.6), 1 / 1.5, nu0, hierarchy.shell_flags(*sh1), parent=0)
    sh2 = (11, 10, 10)
    s2 = Spec(sh2, (8.1, 6.3, 6.2), 0.5, nu0, hierarchy.shell_flags(*sh2), parent=0)
    H, levs, oscs = build_pair([s0, s1, s2], 22)
    assert H.parents == [-1, 0, 0]
    assert H.post_full[(2, 1)].size > 0 and H.post_full[(1, 0)].size > 0
    H.step(3)
    ml.multiscale_step(oscs, 3)
    torch.cuda.synchronize()
    for lev, osc in zip(levs, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5


def test_alpha_one_two_scale_gpu_run_equals_single_scale_gpu_run():
    n = 20
    nu0 = 5e-3
    s0 = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, nu0, np.zeros(n ** 3, np.uint8), periodic=7)
    sh = (9, 8, 10)
    s1 = Spec(sh, (4.0, 6.0, 3.0), 1.0, nu0, hierarchy.shell_flags(*sh), parent=0)
    single, _ = start_both(s0, 30, scalar=False)
    single.step(4)
    lev0, _ = start_both(s0, 30, scalar=False)
    x, y, z = inputs.grid_coords(*sh)
    idx = (x + 4) + n * ((y + 6) + n * (z + 3))
    lev1 = s1.level(False)
    h0, _ = lev0.get_populations(shifted=True)
    lev1.set_populations(h0[:, torch.as_tensor(idx, device="cuda")], shifted=True)
    H = hierarchy.Hierarchy([lev0, lev1], [s0.kinds, s1.kinds], [-1, 0])
    H.step(4)
    torch.cuda.synchronize()
    ref = gpu_pop(single)
    assert rel_err(gpu_pop(lev0), ref) <= 1e-6
    inner = np.flatnonzero(s1.kinds == _capi.FLUID)
    assert rel_err(gpu_pop(lev1)[:, inner], ref[:, idx[inner]]) <= 1e-6


def plume_specs(nx, ny, nz, nu0):
    """Reduced plume scene: walls, inlet disk on x = 0, outflow at x = nx-1,
    sphere; two nested finer boxes around the sphere and its wake
    (alpha = 1.5, 2)."""
    sc = nx / 512.0
    r_sphere = 24.0 * sc
    centre = (160.0 * sc, ny / 2.0, nz / 2.0)
    k0 = inputs.plume_flags(nx, ny, nz)
    s0 = Spec((nx, ny, nz), (0.0, 0.0, 0.0), 1.0, nu0, k0, periodic=0, u_in=(0.05, 0.0, 0.0),
              s_in=1.0)
    specs = [s0]
    boxes = [((centre[0] - 9, 12.0, 10.0), (38.0, 24.0, 28.0), 1 / 1.5),
             ((centre[0] - 6, 16.0, 14.0), (26.0, 16.0, 20.0), 0.5)]
    for i, (org, ext, dx) in enumerate(boxes):
        shape = tuple(int(round(e / dx)) + 1 for e in ext)
        sp = Spec(shape, org, dx, nu0, None, parent=i)
        px, py, pz = sp.positions()
        inner = np.zeros(sp.n, np.uint8)
        inner[(px + 0.5 - centre[0]) ** 2 + (py + 0.5 - centre[1]) ** 2 +
              (pz + 0.5 - centre[2]) ** 2 <= r_sphere ** 2] = _capi.SOLID
        sp.kinds = hierarchy.shell_flags(*shape, inner)
        specs.append(sp)
    return specs


def test_reduced_plume_three_scales_match_oracle():
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    levs, oscs = [], []
    for i, sp in enumerate(specs):
        rho, u, s = smooth_state(sp, 40)       # same physical field on every scale
        u[0] += 0.04
        lev = sp.level(True)
        lev.init_equilibrium(rho, u, s)
        osc = sp.oscale()
        osc.f, osc.g = oracle.init(osc.domain(), rho, u, s=s)
        levs.append(lev)
        oscs.append(osc)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs])
    ml.prepare(oscs)
    for i in range(1, 3):
        for j in range(i):
            np.testing.assert_array_equal(np.sort(H.post_full[(i, j)].astype(np.int64)), oscs[i].post[j])
    H.step(12)
    ml.multiscale_step(oscs, 12)
    torch.cuda.synchronize()
    for lev, osc in zip(levs, oscs):
        assert rel_err(gpu_pop(lev), osc.f) <= 1e-5
        assert np.max(np.abs(gpu_g(lev) - osc.g)) <= 1e-5


def test_reduced_plume_100_reference_steps_at_the_plume_viscosity():
    """The reduced plume (96x48x48, sphere radius 4.5, the same two finer
    boxes at alpha 1.5 and 2) at the plume's viscosity nu0 = 1e-4 (tau0 =
    0.5003: rounding differences are barely damped) over 100 reference
    steps, both sides given the same masks.  Compared per scale: velocity
    relative L2, the largest population error relative to max(|f|, w_i),
    and the smoke scalar."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-4)
    levs, oscs = [], []
    for sp in specs:
        rho, u, s = smooth_state(sp, 41)
        u[0] += 0.04
        lev = sp.level(True)
        lev.init_equilibrium(rho, u, s)
        osc = sp.oscale()
        osc.f, osc.g = oracle.init(osc.domain(), rho, u, s=s)
        levs.append(lev)
        oscs.append(osc)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs])
    ml.prepare(oscs)
    H.step(100)
    ml.multiscale_step(oscs, 100)
    torch.cuda.synchronize()
    for i, (lev, osc) in enumerate(zip(levs, oscs)):
        fluid = osc.flags == 0
        _, ug, sg = lev.read_macro()
        _, uo, so = oracle.macro(osc.domain(), osc.params, osc.f, osc.g)
        ug = ug.double().cpu().numpy()[:, fluid]
        eu = np.linalg.norm(ug - uo[:, fluid]) / np.linalg.norm(uo[:, fluid])
        ep = rel_err(gpu_pop(lev), osc.f)
        es = np.max(np.abs(gpu_g(lev) - osc.g))
        print(f"scale {i}: velocity rel L2 {eu:.2e}, populations {ep:.2e}, scalar {es:.2e}", flush=True)
        assert eu <= 1e-5
        assert ep <= 1e-5
        assert es <= 1e-5


@pytest.mark.parametrize("storage", [F32, F16S])
def test_x_face_staging_gives_bitwise_the_unstaged_result(storage):
    """The prior-mapping of the ghosts on a box's x-faces reads a staged copy
    of the parent's columns: the same corners and weights, so every scale's
    state after several reference steps is bitwise that of the run that
    reads the parent directly."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    states = []
    for stage in (True, False):
        levs = []
        for sp in specs:
            rho, u, s = smooth_state(sp, 40)
            u[0] += 0.04
            lev = Level(*sp.shape, sp.params(), scalar=True, periodic=sp.periodic, flags=sp.kinds,
                        origin=sp.origin, dx=sp.dx, storage=storage)
            lev.init_equilibrium(rho, u, s)
            levs.append(lev)
        H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs],
                                stage_xfaces=stage)
        for i in (1, 2):
            sc = H.c_scales[i]
            assert bool(sc.stage) == stage
            if stage:
                assert sc.n_ghost_xlo == sc.n_ghost_xhi == specs[i].shape[1] * specs[i].shape[2]
                assert (sc.ghost_xlo, sc.ghost_xhi) == (0, specs[i].shape[0] - 1)
        H.step(6)
        torch.cuda.synchronize()
        states.append([(lev.f.cpu().numpy().copy(), lev.g.cpu().numpy().copy()) for lev in levs])
        assert all(lev.count_nonfinite() == 0 for lev in levs)
    for (fa, ga), (fb, gb) in zip(*states):
        np.testing.assert_array_equal(fa, fb)
        np.testing.assert_array_equal(ga, gb)


def _plume_states(storage, **hier_opts):
    """The reduced plume's hierarchy (both finer boxes) and its levels,
    initialised from one smooth field."""
    nx, ny, nz = 96, 48, 48
    specs = plume_specs(nx, ny, nz, 1e-3)
    levs = []
    for sp in specs:
        rho, u, s = smooth_state(sp, 40)
        u[0] += 0.04
        lev = Level(*sp.shape, sp.params(), scalar=True, periodic=sp.periodic, flags=sp.kinds,
                    origin=sp.origin, dx=sp.dx, storage=storage)
        lev.init_equilibrium(rho, u, s)
        levs.append(lev)
    H = hierarchy.Hierarchy(levs, [sp.kinds for sp in specs], [sp.parent for sp in specs], **hier_opts)
    return H, levs


@pytest.mark.parametrize("plates", ["never", "always"])
@pytest.mark.parametrize("storage", [F32, F16S])
def test_tiled_post_mapping_gives_bitwise_the_gathered_result(storage, plates):
    """Post-mapping lists regrouped into tiles (scale 2 -> 1 at ratio 4/3,
    scale 1 -> 0 at 1.5, however sparsely filled; scale 2 -> 0 sits on
    coarse lattice points and the library gathers it), plane tiles or tiles
    lying in the lists' plates, and mapped one tile per workgroup
    through LDS: the same corners, weights and summation order, so every
    scale's state after several reference steps is bitwise that of the
    direct gather."""
    states = []
    for tiles in (True, False):
        H, levs = _plume_states(storage, tile_posts=tiles, tile_min_fill=0, tile_plates=plates)
        n_tiles = {(i, j): H.c_scales[i].n_post_tiles[j] for i in (1, 2) for j in range(i)}
        if tiles:
            assert n_tiles[(2, 1)] > 0 and n_tiles[(1, 0)] > 0
        else:
            assert all(v == 0 for v in n_tiles.values())
        H.step(6)
        torch.cuda.synchronize()
        states.append([(lev.f.cpu().numpy().copy(), lev.g.cpu().numpy().copy()) for lev in levs])
        assert all(lev.count_nonfinite() == 0 for lev in levs)
    for (fa, ga), (fb, gb) in zip(*states):
        np.testing.assert_array_equal(fa, fb)
        np.testing.assert_array_equal(ga, gb)


def test_runs_that_are_not_tiles_give_bitwise_the_gathered_result():
    """Runs of 256 consecutive entries of the box-ordered lists: runs inside
    one plane are staged through LDS, runs that cross planes reach a source
    box larger than the buffer and are gathered directly by the same kernel;
    the last run is partial.  Either way the result is bitwise the plain
    gather's."""
    states = []
    keep = []
    for runs in (True, False):
        H, levs = _plume_states(F32, tile_posts=False)
        if runs:
            for i, j in ((2, 1), (1, 0)):
                n = H.c_scales[i].n_post[j]
                offsets = np.append(np.arange(0, n, 256), n).astype(np.int32)
                t = torch.as_tensor(offsets, device="cuda")
                keep.append(t)
                H.c_scales[i].post_tiles[j] = t.data_ptr()
                H.c_scales[i].n_post_tiles[j] = offsets.size - 1
        H.step(4)
        torch.cuda.synchronize()
        states.append([(lev.f.cpu().numpy().copy(), lev.g.cpu().numpy().copy()) for lev in levs])
    for (fa, ga), (fb, gb) in zip(*states):
        np.testing.assert_array_equal(fa, fb)
        np.testing.assert_array_equal(ga, gb)


@pytest.mark.parametrize("storage", [F32, F16S])
def test_shell_patches_give_bitwise_the_gathered_result(storage):
    """The ghost shells after their x-face entries grouped into patches of
    their faces (one cell deep, 64 x 4 where the parent box fits the
    buffer), each mapped by one workgroup through LDS, at time weights 0, 1
    and in between (the two levels blended on their way into LDS): the same
    corners, weights and summation order, so every scale's state after
    several reference steps is bitwise that of the direct gather."""
    states = []
    for tiles in (True, False):
        H, levs = _plume_states(storage, tile_shells=tiles)
        for i in (1, 2):
            sc = H.c_scales[i]
            assert (sc.n_ghost_tiles > 0) == tiles
        H.step(6)
        torch.cuda.synchronize()
        states.append([(lev.f.cpu().numpy().copy(), lev.g.cpu().numpy().copy()) for lev in levs])
        assert all(lev.count_nonfinite() == 0 for lev in levs)
    for (fa, ga), (fb, gb) in zip(*states):
        np.testing.assert_array_equal(fa, fb)
        np.testing.assert_array_equal(ga, gb)


def test_shell_runs_that_are_not_patches_give_bitwise_the_gathered_result():
    """Runs of 256 consecutive entries of the ghost lists in their plain
    order (each x plane's entries in (z, y) order, then the rest in box
    order): runs inside one face row reach a source box within the shell
    kernel's buffer and are staged through LDS, runs that wrap to the next
    row or face reach a larger box and are gathered directly by the same
    kernel (from the staged copies for the x planes); each part's last run
    is partial.  Either way the result is bitwise the plain gather's."""
    states = []
    keep = []
    for runs in (True, False):
        H, levs = _plume_states(F32, tile_shells=False)
        if runs:
            for i in (1, 2):
                sc = H.c_scales[i]
                bounds = np.cumsum([0, sc.n_ghost_xlo, sc.n_ghost_xhi])
                assert sc.n_ghost_xlo > 0 and sc.n_ghost_xhi > 0
                offsets = np.concatenate([np.arange(a, b, 256) for a, b in
                                          zip(bounds, [bounds[1], bounds[2], sc.n_ghost])]
                                         + [[sc.n_ghost]]).astype(np.int32)
                t = torch.as_tensor(offsets, device="cuda")
                keep.append(t)
                sc.ghost_tiles = t.data_ptr()
                sc.n_ghost_tiles = offsets.size - 1
        H.step(4)
        torch.cuda.synchronize()
        states.append([(lev.f.cpu().numpy().copy(), lev.g.cpu().numpy().copy()) for lev in levs])
    for (fa, ga), (fb, gb) in zip(*states):
        np.testing.assert_array_equal(fa, fb)
        np.testing.assert_array_equal(ga, gb)


def test_vorticity_matches_central_differences():
    """|curl u| (placement of dynamic scales) of an initialised state equals
    central differences of the input field; one-sided at non-periodic faces."""
    n = 20
    rho, u = inputs.taylor_green_3d(n, 0.05)
    for periodic, flags in ((7, None), (0, np.zeros(n ** 3, np.uint8))):
        lev = Level(n, n, n, Params(nu=0.01), periodic=periodic, flags=flags)
        lev.init_equilibrium(rho, u)
        om_t, sp_t = lev.vorticity()
        om = om_t.double().cpu().numpy()
        np.testing.assert_allclose(sp_t.double().cpu().numpy(), np.linalg.norm(u, axis=0),
                                   rtol=0, atol=1e-6)
        U = u.reshape(3, n, n, n)        # [comp, z, y, x]

        def d(a, axis):
            if periodic:
                return (np.roll(a, -1, axis) - np.roll(a, 1, axis)) / 2
            return np.gradient(a, axis=axis, edge_order=1)
        wx = d(U[2], 1) - d(U[1], 0)
        wy = d(U[0], 0) - d(U[2], 2)
        wz = d(U[1], 2) - d(U[0], 1)
        ref = np.sqrt(wx ** 2 + wy ** 2 + wz ** 2).reshape(-1)
        np.testing.assert_allclose(om, ref, rtol=0, atol=1e-6)


def _exchange_gpu(lev_src, lev_dst, cells, w=0.0, lev_b=None):
    import ctypes as C
    cells_t = torch.as_tensor(np.asarray(cells, np.int32), device="cuda")
    lev_src._sync_struct()
    lev_dst._sync_struct()
    fb = None if lev_b is None else lev_b.f.data_ptr()
    gb = None if lev_b is None else lev_b.g.data_ptr()
    _capi.call("cslbm_exchange", C.byref(lev_src.c), lev_src.f.data_ptr(), fb,
               lev_src.g.data_ptr(), gb, float(w), C.byref(lev_dst.c), lev_dst.f.data_ptr(),
               lev_dst.g.data_ptr(), cells_t.data_ptr(), int(cells_t.numel()),
               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()


def test_exchange_on_coincident_lattices_matches_oracle():
    """Fine (spacing 1/2) to coarse with the origins on whole fine cells:
    every target is a fine lattice point (the one-corner path)."""
    n = 20
    coarse = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, 2e-3, np.zeros(n ** 3, np.uint8), periodic=7)
    fshape = (22, 20, 18)
    fine = Spec(fshape, (4.5, 5.0, 3.5), 0.5, 2e-3, hierarchy.shell_flags(*fshape))
    levC, oC = start_both(coarse, 6)
    levF, oF = start_both(fine, 7)
    cells = hierarchy.post_cells(coarse.kinds, coarse.shape, coarse.origin, 1.0, fine.kinds,
                                 fine.shape, fine.origin, fine.dx)
    assert cells.size > 100
    _exchange_gpu(levF, levC, cells)
    fo, go = oC.f.copy(), oC.g.copy()
    oracle.exchange(geom(fine), oF.f, oF.f, 0.0, geom(coarse), cells.astype(np.int64), fo, oF.g,
                    oF.g, go)
    assert rel_err(gpu_pop(levC), fo) <= 1e-6
    assert np.max(np.abs(gpu_g(levC) - go)) <= 2e-7


@pytest.mark.parametrize("s_store,d_store", [(F16S, F16S), (F32, F16S), (F16S, F32)])
def test_exchange_with_binary16_storage_matches_oracle(s_store, d_store):
    """Source and destination in binary16 storage: the oracle takes the
    stored (rounded) source state; the result is within the rounding of its
    own storage."""
    n = 20
    src = Spec((n, n, n), (0.0, 0.0, 0.0), 1.0, 2e-3, np.zeros(n ** 3, np.uint8), periodic=7)
    dshape = (15, 13, 12)
    dst = Spec(dshape, (3.3, 2.6, 7.1), 1 / 1.5, 2e-3, hierarchy.shell_flags(*dshape))
    rho, u, s = smooth_state(src, 8)
    levS = Level(*src.shape, src.params(), storage=s_store, scalar=True, periodic=7)
    levS.init_equilibrium(rho, u, s)
    levD = Level(*dst.shape, dst.params(), storage=d_store, scalar=True, periodic=0,
                 flags=dst.kinds, origin=dst.origin, dx=dst.dx)
    cells = np.arange(dst.n, dtype=np.int32)
    _exchange_gpu(levS, levD, cells)
    hS, gS = levS.get_populations(shifted=True)
    fS = hS.double().cpu().numpy() + W[:, None]
    fo = np.zeros((27, dst.n))
    go = np.zeros((7, dst.n))
    oracle.exchange(geom(src), fS, fS, 0.0, geom(dst), cells.astype(np.int64), fo,
                    gS.double().cpu().numpy(), gS.double().cpu().numpy(), go)
    hD, gD = levD.get_populations(shifted=True)
    got = hD.double().cpu().numpy() + W[:, None]
    if d_store == F32:
        assert rel_err(got, fo) <= 1e-6
    else:
        scale = np.abs(fo - W[:, None]).max(axis=0, keepdims=True)
        assert np.all(np.abs(got - fo) <= 2.0 * 2.0 ** -11 * scale + 2.0 ** -24 + 1e-7 * np.abs(fo))
    assert np.max(np.abs(gD.double().cpu().numpy() - go)) <= 2e-7
