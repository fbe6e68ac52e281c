"""The GPU hierarchy's cell lists (vectorised builder) equal the oracle's
(plain loops): post-mapping targets and ghost shells, bit for bit."""
import numpy as np
import pytest

import oracle
from oracle import multilevel as ml
from paper_1807_02284_amd import hierarchy, inputs


def make(nx, ny, nz, origin, dx, kinds, periodic=0):
    return ml.OScale(nx, ny, nz, dx, origin, oracle.Params(), kinds, periodic=periodic)


@pytest.mark.parametrize("alpha,origin", [(1.5, (3.3, 2.6, 2.2)), (2.0, (4.0, 3.0, 5.5)),
                                          (1.0, (3.0, 2.0, 4.0)), (1.25, (2.9, 3.1, 2.7))])
def test_post_lists_match_oracle(alpha, origin):
    n = 16
    coarse_kinds = np.zeros(n ** 3, np.uint8)
    x, y, z = inputs.grid_coords(n, n, n)
    coarse_kinds[(x == 8) & (y == 8) & (z == 8)] = oracle.SOLID
    fine_shape = (11, 9, 10)
    fine_kinds = hierarchy.shell_flags(*fine_shape)
    fx, fy, fz = inputs.grid_coords(*fine_shape)
    fine_kinds[(fx == 5) & (fy == 4) & (fz == 5)] = oracle.SOLID
    c = make(n, n, n, (0.0, 0.0, 0.0), 1.0, coarse_kinds, periodic=7)
    f = make(*fine_shape, origin, 1.0 / alpha, fine_kinds)
    ref = ml.post_targets(c, f)
    got = hierarchy.post_cells(coarse_kinds, (n, n, n), (0.0, 0.0, 0.0), 1.0,
                               fine_kinds, fine_shape, origin, 1.0 / alpha)
    assert ref.size > 0
    np.testing.assert_array_equal(np.sort(got.astype(np.int64)), ref)
    np.testing.assert_array_equal(np.flatnonzero(fine_kinds == oracle.GHOST), ml.shell_ghosts(f))


@pytest.mark.parametrize("alpha,origin,solid_frac", [(1.5, (3.3, 2.6, 2.2), 0.6), (2.0, (4.0, 3.0, 5.5), 0.85),
                                                     (1.25, (2.9, 3.1, 2.7), 0.3)])
def test_post_lists_match_oracle_when_the_fine_box_is_mostly_solid(alpha, origin, solid_frac):
    """Fine kinds as a brick level's box view has them (most cells SOLID):
    the corner gather must rule out every coarse cell whose stencil touches
    one, as the oracle's cell-by-cell loop does."""
    n = 16
    rng = np.random.default_rng(int(alpha * 100) + int(solid_frac * 10))
    coarse_kinds = np.zeros(n ** 3, np.uint8)
    fine_shape = (13, 11, 12)
    fine_kinds = hierarchy.shell_flags(*fine_shape)
    inner = fine_kinds == 0
    fine_kinds[inner & (rng.random(fine_kinds.size) < solid_frac)] = oracle.SOLID
    c = make(n, n, n, (0.0, 0.0, 0.0), 1.0, coarse_kinds, periodic=7)
    f = make(*fine_shape, origin, 1.0 / alpha, fine_kinds)
    ref = ml.post_targets(c, f)
    got = hierarchy.post_cells(coarse_kinds, (n, n, n), (0.0, 0.0, 0.0), 1.0,
                               fine_kinds, fine_shape, origin, 1.0 / alpha)
    np.testing.assert_array_equal(np.sort(got.astype(np.int64)), ref)


def test_prior_stencil_check_rejects_ghosts_outside_parent():
    n = 8
    kinds = np.zeros(n ** 3, np.uint8)
    fine_shape = (6, 6, 6)
    ghosts = np.flatnonzero(hierarchy.shell_flags(*fine_shape) == oracle.GHOST)
    hierarchy.check_prior_stencils(kinds, (n, n, n), (0, 0, 0), 1.0, 0, fine_shape,
                                   (1.0, 1.0, 1.0), 1.0, ghosts)
    with pytest.raises(ValueError):
        hierarchy.check_prior_stencils(kinds, (n, n, n), (0, 0, 0), 1.0, 0, fine_shape,
                                       (4.5, 1.0, 1.0), 1.0, ghosts)


def test_drop_overwritten_posts_keeps_only_the_last_writer():
    post = {(1, 0): np.array([1, 2, 3, 4]), (2, 0): np.array([3, 4, 5]),
            (2, 1): np.array([7, 8]), (3, 0): np.array([1, 9]), (3, 1): np.array([8]),
            (3, 2): np.array([0])}
    out = hierarchy.drop_overwritten_posts(post, 4)
    assert out[(1, 0)].tolist() == [2]
    assert out[(2, 0)].tolist() == [3, 4, 5]
    assert out[(3, 0)].tolist() == [1, 9]
    assert out[(2, 1)].tolist() == [7]
    assert out[(3, 1)].tolist() == [8]
    assert out[(3, 2)].tolist() == [0]
    # replaying the writes in scale order leaves the same labels
    for lists in (post, out):
        state = {j: np.full(10, -1) for j in range(4)}
        for i in range(1, 4):
            for j in range(i):
                state[j][lists[(i, j)]] = i
        if lists is post:
            full = {j: v.copy() for j, v in state.items()}
    for j in range(4):
        np.testing.assert_array_equal(state[j], full[j])


def _three_scales(n=12):
    rho = np.ones(n ** 3)
    u = inputs.smooth_random_field(n, n, n, 0.04, 77, k_max=2)
    dom = oracle.Domain(n, n, n)
    f0, _ = oracle.init(dom, rho, u)
    nu0 = 2e-3

    def box(nx, ny, nz, origin, dx, nu, parent):
        fl = hierarchy.shell_flags(nx, ny, nz)
        s = ml.OScale(nx, ny, nz, dx, origin, oracle.Params(nu=nu, g_max=0.05), fl, periodic=0,
                      parent=parent)
        return s

    s0 = ml.OScale(n, n, n, 1.0, (0.0, 0.0, 0.0), oracle.Params(nu=nu0, g_max=0.05),
                   np.zeros(n ** 3, np.uint8), periodic=7, f=f0)
    s1 = box(13, 12, 12, (2.0, 2.0, 2.0), 1 / 1.5, nu0 * 1.5, 0)
    s2 = box(12, 10, 10, (3.5, 3.5, 3.5), 0.5, nu0 * 2.0, 1)
    scales = [s0, s1, s2]
    for s in scales[1:]:
        par = scales[s.parent]
        cells = np.arange(s.n)
        s.f = np.zeros((27, s.n))
        oracle.exchange(par.geom(), par.f, par.f, 0.0, s.geom(), cells, s.f)
    ml.prepare(scales)
    return scales


def _siblings(n=12):
    """Two finer scales that are both children of the reference scale, the
    second overlapping the first."""
    rho = np.ones(n ** 3)
    u = inputs.smooth_random_field(n, n, n, 0.04, 78, k_max=2)
    dom = oracle.Domain(n, n, n)
    f0, _ = oracle.init(dom, rho, u)
    nu0 = 2e-3
    s0 = ml.OScale(n, n, n, 1.0, (0.0, 0.0, 0.0), oracle.Params(nu=nu0, g_max=0.05),
                   np.zeros(n ** 3, np.uint8), periodic=7, f=f0)
    s1 = ml.OScale(10, 10, 10, 1 / 1.5, (1.3, 2.4, 2.6), oracle.Params(nu=nu0 * 1.5, g_max=0.05),
                   hierarchy.shell_flags(10, 10, 10), periodic=0, parent=0)
    s2 = ml.OScale(9, 9, 9, 0.5, (5.1, 3.3, 3.2), oracle.Params(nu=nu0 * 2.0, g_max=0.05),
                   hierarchy.shell_flags(9, 9, 9), periodic=0, parent=0)
    scales = [s0, s1, s2]
    for s in scales[1:]:
        s.f = np.zeros((27, s.n))
        oracle.exchange(s0.geom(), s0.f, s0.f, 0.0, s.geom(), np.arange(s.n), s.f)
    ml.prepare(scales)
    return scales


def test_posts_read_by_a_later_sibling_are_kept_whole():
    """With sibling scales (both children of the reference), the second's
    prior-mappings read reference cells that the first post-maps: its list
    into the reference must stay whole.  The oracle run with the kept lists
    equals the full-list run bit for bit; dropping by the chain rule would
    not."""
    full = _siblings()
    lists = {(i, j): full[i].post[j] for i in range(1, 3) for j in range(i)}
    assert lists[(2, 0)].size > 0 and lists[(1, 0)].size > 0
    assert np.intersect1d(lists[(1, 0)], lists[(2, 0)]).size > 0
    kept = hierarchy.drop_overwritten_posts(lists, 3, [-1, 0, 0])
    chain = hierarchy.drop_overwritten_posts(lists, 3)
    np.testing.assert_array_equal(kept[(1, 0)], lists[(1, 0)])
    assert chain[(1, 0)].size < lists[(1, 0)].size
    ml.multiscale_step(full, 2)
    for red_lists, same in ((kept, True), (chain, False)):
        red = _siblings()
        for (i, j), cells in red_lists.items():
            red[i].post[j] = np.asarray(cells, np.int64)
        ml.multiscale_step(red, 2)
        equal = all(np.array_equal(a.f, b.f) for a, b in zip(full, red))
        assert equal == same


def test_dropping_overwritten_post_cells_leaves_the_oracle_state_bit_identical():
    """Three scales (alpha 1.5 and 2, nested): the oracle's Algorithm-1 run
    with the reduced post-mapping lists equals the run with the full lists
    bit for bit, after 2 reference steps."""
    full = _three_scales()
    red = _three_scales()
    lists = {(i, j): red[i].post[j] for i in range(1, 3) for j in range(i)}
    dropped = hierarchy.drop_overwritten_posts(lists, 3)
    assert dropped[(1, 0)].size < lists[(1, 0)].size
    for (i, j), cells in dropped.items():
        red[i].post[j] = cells.astype(np.int64)
    ml.multiscale_step(full, 2)
    ml.multiscale_step(red, 2)
    for a, b in zip(full, red):
        np.testing.assert_array_equal(a.f, b.f)


def test_kept_cells_pair_the_same_lattice_points_of_two_boxes():
    from types import SimpleNamespace

    dx = 1 / 1.5

    def box(i0, shape):
        c = SimpleNamespace(dx=dx, origin=tuple(i * dx for i in i0))
        kinds = hierarchy.shell_flags(*shape)
        return SimpleNamespace(c=c, nx=shape[0], ny=shape[1], nz=shape[2]), kinds

    old, ko = box((10, 4, 7), (12, 9, 8))
    new, kn = box((14, 2, 9), (11, 10, 9))
    src, dst = hierarchy.kept_cells(old, ko, new, kn)
    assert src.size > 0
    # brute force over the new box
    pairs = set()
    for c in np.flatnonzero(kn == hierarchy.FLUID):
        x, y, z = c % 11, (c // 11) % 10, c // 110
        g = (x + 14, y + 2, z + 9)
        lx, ly, lz = g[0] - 10, g[1] - 4, g[2] - 7
        if 0 <= lx < 12 and 0 <= ly < 9 and 0 <= lz < 8:
            co = lx + 12 * (ly + 9 * lz)
            if ko[co] == hierarchy.FLUID:
                pairs.add((co, c))
    assert pairs == set(zip(src.tolist(), dst.tolist()))


def test_region_box_is_the_dilated_clipped_bounding_box_of_both_thresholds():
    rng = np.random.default_rng(5)
    shape = (30, 20, 16)
    n = int(np.prod(shape))
    x, y, z = inputs.grid_coords(*shape)
    om = rng.random(n) * 1e-3
    sp = rng.random(n) * 1e-2
    blob = (np.abs(x - 17) < 5) & (np.abs(y - 9) < 4) & (np.abs(z - 6) < 3)
    om[blob] += 0.01
    sp[blob] += 0.05
    sp[(x == 20) & (y == 10) & (z == 7)] = 0.0          # fails the speed threshold
    om[(x == 3) & (y == 3) & (z == 3)] = 1.0            # passes vorticity, not speed
    box = hierarchy.region_box(om, sp, shape, (5e-3, 2e-2), 2, [2, 2, 2], [27, 17, 13])
    sel = (om > 5e-3) & (sp > 2e-2)
    lo = [max(x[sel].min() - 2, 2), max(y[sel].min() - 2, 2), max(z[sel].min() - 2, 2)]
    hi = [min(x[sel].max() + 2, 27), min(y[sel].max() + 2, 17), min(z[sel].max() + 2, 13)]
    assert box == (lo, hi)
    assert hierarchy.region_box(om, sp, shape, (1.0, 1.0), 2, [2, 2, 2], [27, 17, 13]) is None
    # a region thinner than 3 cells after clipping is dropped
    assert hierarchy.region_box(om, sp, shape, (5e-3, 2e-2), 0, [2, 2, 2], [27, 17, 6]) is None


@pytest.mark.parametrize("ratio", [4.0 / 3.0, 1.5, 2.0, 3.2])
def test_plate_tile_runs_partition_a_nested_shell_into_filled_tiles_whose_source_box_fits(ratio):
    """Plate tiles of the cells between two nested boxes (plates two cells
    thick on all six sides, as the part of scale 1 that scale 2 does not
    overwrite): a permutation of the list, at most 256 entries a run, each
    run's cells in box order, every run's source box (the corner b + 1 only
    where the fraction is not 0) within the kernel's buffer, and tiles far
    fuller than plane tiles of the same list."""
    shape = (150, 90, 80)
    nx, ny, nz = shape
    x, y, z = inputs.grid_coords(*shape)
    outer = (x >= 3) & (x <= 146) & (y >= 4) & (y <= 85) & (z >= 2) & (z <= 77)
    inner = (x >= 5) & (x <= 144) & (y >= 6) & (y <= 83) & (z >= 4) & (z <= 75)
    cells = np.flatnonzero(outer & ~inner).astype(np.int32)
    out, runs = hierarchy.plate_tile_runs(cells, shape, ratio)
    np.testing.assert_array_equal(np.sort(out), np.sort(cells))
    assert runs[0] == 0 and runs[-1] == cells.size
    sizes = np.diff(runs)
    assert np.all(sizes >= 1) and np.all(sizes <= hierarchy.POST_RUN)
    fine_dx = 1.0 / ratio
    for a, b in zip(runs[:-1], runs[1:]):
        c = out[a:b].astype(np.int64)
        assert np.all(np.diff(c) > 0)
        vol = 1
        for p in (c % nx, (c // nx) % ny, c // (nx * ny)):
            q = (p * 1.0 - 0.25) / fine_dx
            base = np.floor(q)
            top = np.where(q - base != 0.0, base + 1, base)
            vol *= int(top.max() - base.min() + 1)
        assert vol <= hierarchy.POST_TILE_BUFFER, (ratio, vol)
    _, plane = hierarchy.post_tile_runs(cells, shape, ratio)
    assert cells.size / sizes.size > 2.0 * cells.size / (plane.size - 1)


@pytest.mark.parametrize("ratio,origin", [(0.75, (3.3, 2.6, 2.2)), (2 / 3, (0.4, 1.1, 0.7)),
                                          (0.5, (1.25, 0.75, 0.25))])
def test_shell_tile_runs_partition_a_ghost_shell_into_full_patches_whose_source_box_fits(ratio, origin):
    """Patch runs of a one-cell ghost shell, an x plane (which reads a
    staged copy) apart from the rest: a permutation of the list, at most
    256 entries a run, each run's cells in box order, every run's parent
    box (the corner b + 1 only where the fraction is not 0, as the kernel
    does) within the shell kernel's buffer, and runs mostly full."""
    shape = (150, 61, 47)
    nx, ny, nz = shape
    g = np.flatnonzero(hierarchy.shell_flags(*shape) == hierarchy.GHOST)
    gx = g % nx
    cells = g[(gx != 0) & (gx != nx - 1)].astype(np.int32)
    out, runs = hierarchy.shell_tile_runs(cells, shape, ratio)
    lo = g[gx == 0].astype(np.int32)
    out_lo, runs_lo = hierarchy.shell_tile_runs(lo, shape, ratio, xface=True)
    assert lo.size / (runs_lo.size - 1) >= 150
    _check_shell_runs(out_lo, runs_lo, lo, shape, ratio, origin)
    _check_shell_runs(out, runs, cells, shape, ratio, origin)


def _check_shell_runs(out, runs, cells, shape, ratio, origin):
    nx, ny, nz = shape
    np.testing.assert_array_equal(np.sort(out), np.sort(cells))
    assert runs[0] == 0 and runs[-1] == cells.size
    sizes = np.diff(runs)
    assert np.all(sizes >= 1) and np.all(sizes <= hierarchy.POST_RUN)
    assert cells.size / sizes.size >= 150
    for a, b in zip(runs[:-1], runs[1:]):
        c = out[a:b].astype(np.int64)
        assert np.all(np.diff(c) > 0)
        xyz = (c % nx, (c // nx) % ny, c // (nx * ny))
        vol = 1
        for p, o in zip(xyz, origin):
            q = o + p * ratio
            base = np.floor(q)
            top = np.where(q - base != 0.0, base + 1, base)
            vol *= int(top.max() - base.min() + 1)
        assert vol <= hierarchy.SHELL_TILE_BUFFER, (ratio, vol)


def test_plate_tiles_fit_the_buffer_and_lie_two_cells_deep():
    """The plate tile of each orientation: two cells deep along its axis, at
    most 256 cells, source box within the buffer, and no larger tile of the
    same depth would fit."""
    for ratio in (1.0, 4.0 / 3.0, 1.5, 2.0, 3.2):
        for axis in (0, 1, 2):
            t = hierarchy._plate_tile(axis, ratio)
            assert t[axis] == 2 and t[0] * t[1] * t[2] <= hierarchy.POST_RUN
            assert hierarchy._tile_source_cells(t, ratio) <= hierarchy.POST_TILE_BUFFER
            a, b = [t[d] for d in range(3) if d != axis]
            for grown in ((a + 1, b), (a, b + 1)):
                if grown[0] * grown[1] * 2 > hierarchy.POST_RUN:
                    continue
                g = list(grown)
                g.insert(axis, 2)
                assert (hierarchy._tile_source_cells(g, ratio) > hierarchy.POST_TILE_BUFFER
                        or g[0] * g[1] * g[2] <= t[0] * t[1] * t[2])


@pytest.mark.parametrize("ratio,origin", [(4 / 3, (3.3, 2.6, 2.2)), (1.5, (0.4, 1.1, 0.7)),
                                          (2.0, (1.25, 0.75, 0.25)), (3.2, (0.3, 0.9, 1.6))])
def test_post_tile_runs_partition_the_list_into_plane_tiles_whose_source_box_fits(ratio, origin):
    """Runs of the tiled post-mapping: a permutation of the list, at most 256
    entries a run, each run inside one plane with its cells in box order,
    and the source cells its trilinear stencils reach (the corner b + 1 only
    where the fraction is not 0, as the kernel does) fit the kernel's
    buffer, so no tile falls back to the direct gather."""
    shape = (70, 33, 9)
    nx, ny, nz = shape
    rng = np.random.default_rng(3)
    x, y, z = inputs.grid_coords(*shape)
    keep = (x >= 3) & (x < 61) & (y >= 2) & (y < 31) & (rng.random(x.size) > 0.1)
    cells = np.flatnonzero(keep).astype(np.int32)
    out, runs = hierarchy.post_tile_runs(cells, shape, ratio)
    np.testing.assert_array_equal(np.sort(out), np.sort(cells))
    assert runs[0] == 0 and runs[-1] == cells.size
    sizes = np.diff(runs)
    assert np.all(sizes >= 1) and np.all(sizes <= hierarchy.POST_RUN)
    fine_dx = 1.0 / ratio
    for a, b in zip(runs[:-1], runs[1:]):
        c = out[a:b].astype(np.int64)
        assert np.all(np.diff(c) > 0)
        cx, cy, cz = c % nx, (c // nx) % ny, c // (nx * ny)
        assert np.all(cz == cz[0])
        vol = 1
        for p, o in ((cx, origin[0]), (cy, origin[1]), (cz, origin[2])):
            q = (p * 1.0 - o) / fine_dx
            base = np.floor(q)
            top = np.where(q - base != 0.0, base + 1, base)
            vol *= int(top.max() - base.min() + 1)
        assert vol <= hierarchy.POST_TILE_BUFFER, (ratio, vol)
