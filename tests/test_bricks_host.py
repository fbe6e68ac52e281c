"""Host logic of sparse brick storage: the storage layout (brick table,
brick coordinates, storage -> box index map), the ghost layer that
``brick_kinds`` puts between the fluid and the bricks that are not stored,
and the C ABI's checks of brick levels (no GPU needed)."""
import ctypes as C

import numpy as np

from paper_1807_02284_amd import _capi, hierarchy
from paper_1807_02284_amd.level import brick_layout
from test_capi_abi import make_level


def test_brick_layout_is_a_bijection_onto_the_stored_bricks():
    nx, ny, nz = 24, 16, 32
    rng = np.random.default_rng(2)
    mask = rng.random((nz // 8, ny // 8, nx // 8)) < 0.6
    table, origin, dense = brick_layout(mask, nx, ny, nz)
    nb = int(mask.sum())
    assert origin.size == 3 * nb and dense.size == 512 * nb
    assert np.unique(dense).size == dense.size
    # every storage index lies in its own brick, x fastest inside the brick
    x, y, z = dense % nx, (dense // nx) % ny, dense // (nx * ny)
    b = np.arange(dense.size) // 512
    o = origin.reshape(-1, 3)
    assert np.array_equal(x // 8, o[b, 0]) and np.array_equal(y // 8, o[b, 1])
    assert np.array_equal(z // 8, o[b, 2])
    l = np.arange(dense.size) % 512
    assert np.array_equal(x % 8 + 8 * (y % 8) + 64 * (z % 8), l)
    # the table points each stored brick at its index, the others at -1
    bricks = (x // 8) + (nx // 8) * ((y // 8) + (ny // 8) * (z // 8))
    assert np.array_equal(table[bricks], b)
    assert np.all(table[~mask.reshape(-1)] == -1)


def test_brick_kinds_keep_every_fluid_neighbourhood_stored():
    shape = (32, 24, 16)
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    region = (x - 15.5) ** 2 + (y - 11.0) ** 2 + (z - 7.0) ** 2 <= 7.5 ** 2
    solid = (x - 15.5) ** 2 + (y - 11.0) ** 2 + (z - 7.0) ** 2 <= 2.0 ** 2
    bricks, kinds = hierarchy.brick_kinds(region, solid)
    assert np.array_equal(bricks, region.reshape(2, 8, 3, 8, 4, 8).any(axis=(1, 3, 5)))
    k = kinds.reshape(nz, ny, nx)
    stored = bricks.repeat(8, 0).repeat(8, 1).repeat(8, 2)
    assert np.all(k[~stored] == _capi.SOLID)
    assert np.all(k[region & ~solid & stored] != _capi.SOLID)   # the region is covered
    fl = np.argwhere(k == _capi.FLUID)
    assert fl.size
    for d in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T:
        nb = fl + d
        assert np.all((nb >= 0).all(axis=1) & (nb < [nz, ny, nx]).all(axis=1))
        assert np.all(stored[nb[:, 0], nb[:, 1], nb[:, 2]])
    # a GHOST cell is a stored cell with a neighbour outside the stored bricks or the box
    gh = np.argwhere(k == _capi.GHOST)
    pad = np.pad(stored, 1, constant_values=False)
    outside = np.zeros(len(gh), bool)
    for d in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T:
        q = gh + d + 1
        outside |= ~pad[q[:, 0], q[:, 1], q[:, 2]]
    assert np.all(outside)


def test_brick_level_argument_checks():
    lib = _capi.load()
    L = make_level(nx=16, ny=16, nz=16, periodic=0, flags=0x9000, brick_table=0xA000,
                   brick_origin=0xB000, n_bricks=3)
    L.plane = 4096
    assert lib.cslbm_step(C.byref(make_level(nx=12, ny=16, nz=16, periodic=0, flags=0x9000,
                                             brick_table=0xA000, brick_origin=0xB000, n_bricks=1)),
                          1, None) == _capi.ERR_SHAPE
    assert lib.cslbm_step(C.byref(make_level(nx=16, ny=16, nz=16, periodic=0, flags=0x9000,
                                             brick_table=0xA000, brick_origin=0xB000, n_bricks=9, plane=8192)),
                          1, None) == _capi.ERR_ARG
    periodic = make_level(nx=16, ny=16, nz=16, periodic=1, flags=0x9000, brick_table=0xA000,
                          brick_origin=0xB000, n_bricks=3, plane=8192)
    assert lib.cslbm_step(C.byref(periodic), 1, None) == _capi.ERR_UNSUPPORTED
    forced = make_level(nx=16, ny=16, nz=16, periodic=0, flags=0x9000, brick_table=0xA000,
                        brick_origin=0xB000, n_bricks=3, force=0xC000, plane=8192)
    assert lib.cslbm_step(C.byref(forced), 1, None) == _capi.ERR_UNSUPPORTED
    no_flags = make_level(nx=16, ny=16, nz=16, periodic=0, brick_table=0xA000,
                          brick_origin=0xB000, n_bricks=3, plane=8192)
    assert lib.cslbm_step(C.byref(no_flags), 1, None) < 0
    vort = lib.cslbm_vorticity
    assert vort(C.byref(L), 0xD000, None, None) == _capi.ERR_UNSUPPORTED


def _plume_like_field(shape, centre, radius, jet_r):
    """A smooth stand-in for the plume's |curl u| and |u|: a jet shear layer
    along x and a wake cone behind a sphere."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((y + 0.5 - ny / 2) ** 2 + (z + 0.5 - nz / 2) ** 2)
    speed = 0.05 * np.exp(-np.maximum(r - jet_r, 0.0) ** 2 / 8.0)
    omega = 0.012 * np.exp(-(r - jet_r) ** 2 / 6.0)
    d = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    wake = (x > centre[0]) & (r < radius + 0.3 * (x - centre[0]))
    omega = np.where(wake | (d < radius + 3), np.maximum(omega, 0.01), omega)
    return omega.reshape(-1), speed.reshape(-1)


def test_brick_regions_of_a_plume_like_flow_nest_on_fluid():
    """The brick construction of the plume benchmark at 128x64x64: every
    scale's ghost stencils lie on its parent's FLUID cells (the sphere is
    taken into the regions whole), and the bricks store fewer cells than
    the regions' bounding boxes."""
    shape = (128, 64, 64)
    nx, ny, nz = shape
    from paper_1807_02284_amd import inputs
    centre, radius = (40.0, 32.0, 32.0), 6.0
    kinds0 = inputs.plume_flags(nx, ny, nz, sphere_center=centre, sphere_radius=radius)
    omega, speed = _plume_like_field(shape, centre, radius, 8.0)

    def sphere(px, py, pz):
        return (px + 0.5 - centre[0]) ** 2 + (py + 0.5 - centre[1]) ** 2 + (pz + 0.5 - centre[2]) ** 2 \
            <= radius ** 2

    alphas = (1.5, 2.0)
    regions = hierarchy.brick_regions(omega, speed, kinds0, shape, ((2e-3, 0.01), (8e-3, 0.02)),
                                      alphas)
    assert len(regions) == 2
    parent = (kinds0, shape, (0.0, 0.0, 0.0), 1.0)
    for region, alpha in zip(regions, alphas):
        lo, hi, fn = hierarchy.region_box_fn(region)
        shp, origin, dx, bricks, kinds = hierarchy.brick_scale_layout(lo, hi, alpha, fn, sphere)
        ghosts = np.flatnonzero(kinds == hierarchy.GHOST)
        hierarchy.check_prior_stencils(parent[0], parent[1], parent[2], parent[3], 0, shp, origin,
                                       dx, ghosts)
        assert bricks.sum() * 512 < np.prod(shp)
        parent = (kinds, shp, origin, dx)


def test_cube_morphology_equals_iterated_3x3x3_structure():
    """Dilation and erosion by a cube of half-width r (three 1-D max-pools)
    equal scipy's binary morphology with the 3x3x3 structure iterated r
    times, cells outside the array counting as False."""
    import torch
    from scipy import ndimage
    rng = np.random.default_rng(17)
    cube = np.ones((3, 3, 3), bool)
    for trial in range(12):
        shape = tuple(int(v) for v in rng.integers(4, 26, 3))
        m = rng.random(shape) < rng.uniform(0.02, 0.9)
        r = int(rng.integers(1, 6))
        t = torch.as_tensor(m)
        np.testing.assert_array_equal(hierarchy._cube_dilate(t, r).numpy(),
                                      ndimage.binary_dilation(m, structure=cube, iterations=r))
        np.testing.assert_array_equal(hierarchy._cube_erode(t, r).numpy(),
                                      ndimage.binary_erosion(m, structure=cube, iterations=r))


def test_storage_of_inverts_the_layout_through_the_brick_table():
    """Box index -> storage index through the brick table equals the inverse
    of the layout's storage -> box map (-1 for cells of unstored bricks)."""
    import types
    from paper_1807_02284_amd.level import Level
    rng = np.random.default_rng(23)
    nx, ny, nz = 24, 16, 32
    mask = rng.random((nz // 8, ny // 8, nx // 8)) < 0.5
    mask.reshape(-1)[0] = True
    table, origin, dense_index = brick_layout(mask, nx, ny, nz)
    lev = types.SimpleNamespace(nx=nx, ny=ny, nz=nz, dense_index=dense_index, _table=table)
    inv = np.full(nx * ny * nz, -1, np.int64)
    inv[dense_index] = np.arange(dense_index.size)
    cells = np.arange(nx * ny * nz)
    np.testing.assert_array_equal(Level.storage_of(lev, cells), inv)
    import pytest
    with pytest.raises(ValueError):
        Level.storage_of(lev, np.array([nx * ny * nz]))
