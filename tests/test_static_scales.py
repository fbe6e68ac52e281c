"""Static scale construction (section "Scale construction": distance map of
the geometry quantised into scales, soft-shadow wake behind objects lit by
the inlet).  Host logic only; the paper fixes no numbers, so these check
the construction against closed forms and brute force ("parity unpinned"
beyond that)."""
import numpy as np

from paper_1807_02284_amd import _capi, hierarchy, inputs


def sphere_kinds(shape, centre, radius):
    x, y, z = inputs.grid_coords(*shape)
    k = np.zeros(x.size, np.uint8)
    r2 = (x + 0.5 - centre[0]) ** 2 + (y + 0.5 - centre[1]) ** 2 + (z + 0.5 - centre[2]) ** 2
    k[r2 <= radius ** 2] = _capi.SOLID
    return k


def test_distance_to_the_faces_of_an_empty_box():
    shape = (20, 16, 12)
    x, y, z = inputs.grid_coords(*shape)
    d = hierarchy.object_distance(np.zeros(x.size, np.uint8), shape, periodic=0)
    expect = np.minimum.reduce([x + 1, shape[0] - x, y + 1, shape[1] - y, z + 1, shape[2] - z])
    np.testing.assert_allclose(d, expect.astype(float))


def test_distance_to_a_solid_sphere_is_the_nearest_solid_cell():
    shape = (18, 14, 12)
    kinds = sphere_kinds(shape, (9, 7, 6), 2.5)
    d = hierarchy.object_distance(kinds, shape, periodic=7)
    x, y, z = inputs.grid_coords(*shape)
    solid = np.flatnonzero(kinds == _capi.SOLID)
    brute = np.sqrt(np.min((x[:, None] - x[solid]) ** 2 + (y[:, None] - y[solid]) ** 2 +
                           (z[:, None] - z[solid]) ** 2, axis=1))
    inner = (x > 2) & (x < 15) & (y > 2) & (y < 11) & (z > 2) & (z < 9)
    np.testing.assert_allclose(d[inner], brute[inner])


def test_shadow_of_a_sphere_behind_a_small_inlet_has_an_umbra_on_the_axis():
    shape = (64, 32, 32)
    kinds = sphere_kinds(shape, (24, 16, 16), 6.0)
    sh = hierarchy.wake_shadow(kinds, shape, (16.0, 16.0), 3.0, samples=16, coarsen=2)
    x, y, z = inputs.grid_coords(*shape)
    on_axis = (np.abs(y + 0.5 - 16) < 2) & (np.abs(z + 0.5 - 16) < 2)
    assert np.all(sh[on_axis & (x >= 34) & (x < 60)] == 1.0)           # umbra downstream
    assert np.all(sh[x < 16] == 0.0)                                     # lit upstream
    off = (np.abs(y + 0.5 - 16) > 13) & (x < 28)
    assert np.all(sh[off] == 0.0)                                        # lit off axis
    pen = sh[~on_axis & (x > 40)]
    assert np.any((pen > 0.0) & (pen < 1.0))                             # a penumbra exists


def test_static_levels_and_boxes_refine_around_the_object_and_its_wake():
    shape = (96, 48, 48)
    centre, radius = (30, 24, 24), 5.0
    kinds = sphere_kinds(shape, centre, radius)
    lv = hierarchy.static_levels(kinds, shape, 3, 8.0, periodic=7, inlet_center=(24.0, 24.0),
                                 inlet_radius=3.0, shadow_coarsen=2)
    assert lv.max() == 2 and np.all(lv[kinds == _capi.SOLID] == 0)
    boxes = hierarchy.static_boxes(lv, shape, 3)
    assert len(boxes) == 2
    (lo1, hi1), (lo2, hi2) = boxes
    # nested, and the finest box holds the sphere
    assert all(lo1[a] + 2 <= lo2[a] and hi2[a] <= hi1[a] - 2 for a in range(3))
    assert lo2[0] <= centre[0] - radius and hi2[0] >= centre[0] + radius
    # the wake stretches the boxes downstream more than upstream
    assert hi1[0] - centre[0] > centre[0] - lo1[0]
