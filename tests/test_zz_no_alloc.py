"""The allocation-free conservation call (cslbm_conserved_f64_noalloc)
against cslbm_conserved_f64 through the C ABI: the same kernels and
reduction order, so the totals are bitwise equal.  Two calls in a row, the
second on a smaller level, check that the library-held scratch is reused
correctly."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1807_02284_amd import _capi, inputs
from paper_1807_02284_amd.level import F16S, F32, Level, Params, _stream_handle

pytestmark = pytest.mark.gpu


def totals_noalloc(lev: Level) -> np.ndarray:
    out = torch.full((5,), float("nan"), dtype=torch.float64, device=lev.device)
    lev._sync_struct()
    _capi.call("cslbm_conserved_f64_noalloc", C.byref(lev.c), C.c_void_p(out.data_ptr()),
               _stream_handle())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def make_level(n, seed, storage, flags=False):
    nx, ny, nz = n
    kinds = None
    if flags:
        kinds = np.zeros(nx * ny * nz, np.uint8)
        x, y, z = inputs.grid_coords(nx, ny, nz)
        kinds[(x == 0) | (x == nx - 1)] = _capi.SOLID
    lev = Level(nx, ny, nz, Params(nu=0.01, tau_s=0.6), storage=storage, scalar=True,
                periodic=6 if flags else 7, flags=kinds)
    cells = nx * ny * nz
    rho = 1.0 + 0.02 * inputs.perturbation(cells, seed)
    u = 0.05 * inputs.perturbation((3, cells), seed + 1)
    s = 0.5 + 0.5 * inputs.perturbation(cells, seed + 2)
    lev.init_equilibrium(rho, u, s)
    lev.step(2)
    return lev


@pytest.mark.parametrize("storage", [F32, F16S])
def test_noalloc_totals_equal_the_allocating_call_on_two_calls_in_a_row(storage):
    torch.cuda.set_device(0)
    big = make_level((70, 33, 21), 5, storage, flags=True)
    small = make_level((9, 7, 5), 9, storage)
    for lev in (big, small):
        print(f"noalloc totals: storage {storage}, shape {(lev.nx, lev.ny, lev.nz)}", flush=True)
        want = lev.conserved()
        got = totals_noalloc(lev)
        assert np.isfinite(got).all()
        np.testing.assert_array_equal(got, want)
