"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds workloads only (velocity fields, cell-kind masks, noise) and
none of the lattice Boltzmann arithmetic: the conversion of (rho, u) into
populations is done separately by each implementation.  Arrays are float64
numpy, fields in ``[component][cell]`` layout with cell = x + nx*(y + ny*z).
"""
from __future__ import annotations

import numpy as np

# cell kinds (one byte per cell), identical in every implementation
FLUID, SOLID, INLET, OUTFLOW, GHOST = 0, 1, 2, 3, 4


def grid_coords(nx: int, ny: int, nz: int):
    """Integer coordinate arrays (x, y, z), each flattened with x fastest."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def taylor_green_2d(nx: int, ny: int, nz: int, u0: float):
    """2D Taylor-Green vortex extruded along z, uniform rho = 1:
    u = u0 cos(kx x) sin(ky y), v = -u0 sin(kx x) cos(ky y), w = 0, with one
    wavelength per box side.  Velocity amplitude decays as exp(-nu (kx^2+ky^2) t)."""
    x, y, _ = grid_coords(nx, ny, nz)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    u = np.zeros((3, x.size))
    u[0] = u0 * np.cos(kx * x) * np.sin(ky * y)
    u[1] = -u0 * np.sin(kx * x) * np.cos(ky * y)
    return np.ones(x.size), u


def taylor_green_3d(n: int, u0: float):
    """3D Taylor-Green initial field (no closed-form decay): u = u0 sin x cos y
    cos z, v = -u0 cos x sin y cos z, w = 0 on an n^3 periodic box."""
    x, y, z = grid_coords(n, n, n)
    k = 2 * np.pi / n
    u = np.zeros((3, x.size))
    u[0] = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    return np.ones(x.size), u


def shear_wave(nx: int, ny: int, nz: int, u0: float):
    """u_x = u0 sin(2 pi y / ny): decays as exp(-nu k^2 t)."""
    _, y, _ = grid_coords(nx, ny, nz)
    u = np.zeros((3, y.size))
    u[0] = u0 * np.sin(2 * np.pi * y / ny)
    return np.ones(y.size), u


def turbulence(n: int, k_min: int = 2, k_max: int = 32, u_rms: float = 0.04,
               seed: int = 1807, per_component: bool = True):
    """Random solenoidal velocity on an n^3 periodic box with E(k) ~ k^(-5/3)
    over integer wavevectors k_min <= |k| <= k_max.

    Complex Gaussian Fourier coefficients with amplitude |k|^(-11/6) (so the
    shell energy goes as k^2 |k|^(-11/3) = k^(-5/3)), projected onto the
    divergence-free subspace, transformed with irfftn and scaled so that the
    rms of each component is u_rms (or |u|_rms = u_rms if per_component is
    False).  numpy PCG64 with the given seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.fft.rfftfreq(n, d=1.0 / n)
    KX, KY, KZ = np.meshgrid(k1, k1, kr, indexing="ij")      # axes (x, y, z)
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = (kk >= k_min) & (kk <= k_max)
    amp = np.zeros_like(kk)
    amp[shell] = kk[shell] ** (-11.0 / 6.0)
    coef = []
    for _ in range(3):
        c = rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape)
        coef.append(c * amp)
    ksafe = np.where(kk > 0, kk, 1.0)
    kdotc = (KX * coef[0] + KY * coef[1] + KZ * coef[2]) / ksafe ** 2
    coef = [coef[0] - KX * kdotc, coef[1] - KY * kdotc, coef[2] - KZ * kdotc]
    vel = [np.fft.irfftn(c, s=(n, n, n), axes=(0, 1, 2)) for c in coef]   # [x, y, z]
    vel = np.stack(vel)                                   # [3, x, y, z]
    vel -= vel.mean(axis=(1, 2, 3), keepdims=True)
    if per_component:
        vel *= u_rms / np.sqrt(np.mean(vel ** 2, axis=(1, 2, 3), keepdims=True))
    else:
        vel *= u_rms / np.sqrt(np.mean(np.sum(vel ** 2, axis=0)))
    # reorder to [component][cell] with x fastest: index (z, y, x)
    u = vel.transpose(0, 3, 2, 1).reshape(3, -1)
    return np.ones(n ** 3), np.ascontiguousarray(u)


def perturbation(shape, seed: int, scale: float = 1.0):
    """Seeded uniform noise in [-scale, scale), float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=shape)


def plume_flags(nx: int, ny: int, nz: int, inlet_center=None, inlet_radius=None,
                sphere_center=None, sphere_radius=None):
    """Cell kinds of the plume scene: walls (solid) on the y and z faces and on
    the x = 0 face outside the inlet disk, an inlet disk on the x = 0 face, a
    solid sphere (cell centre inside => solid) and an outflow plane at
    x = nx - 1.  Defaults scale the 512x256x256 scene (disk radius 32 at
    (128, 128), sphere radius 24 at (160, 128, 128))."""
    s = nx / 512.0
    if inlet_center is None:
        inlet_center = (ny / 2.0, nz / 2.0)
    if inlet_radius is None:
        inlet_radius = 32.0 * s
    if sphere_center is None:
        sphere_center = (160.0 * s, ny / 2.0, nz / 2.0)
    if sphere_radius is None:
        sphere_radius = 24.0 * s
    x, y, z = grid_coords(nx, ny, nz)
    fl = np.full(x.size, FLUID, dtype=np.uint8)
    wall = (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    disk = (x == 0) & ((y + 0.5 - inlet_center[0]) ** 2 + (z + 0.5 - inlet_center[1]) ** 2
                       <= inlet_radius ** 2)
    fl[(x == 0) & ~disk] = SOLID
    fl[disk & ~wall] = INLET
    fl[x == nx - 1] = OUTFLOW
    fl[wall] = SOLID
    r2 = ((x + 0.5 - sphere_center[0]) ** 2 + (y + 0.5 - sphere_center[1]) ** 2 +
          (z + 0.5 - sphere_center[2]) ** 2)
    fl[r2 <= sphere_radius ** 2] = SOLID
    return fl


def gaussian_blob(nx: int, ny: int, nz: int, center, sigma: float):
    """s = exp(-r^2 / (2 sigma^2)) on cell centres (periodic distance)."""
    x, y, z = grid_coords(nx, ny, nz)
    d = []
    for coord, c, n in ((x, center[0], nx), (y, center[1], ny), (z, center[2], nz)):
        dd = np.abs(coord - c)
        d.append(np.minimum(dd, n - dd))
    r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
    return np.exp(-r2 / (2.0 * sigma ** 2))


def smooth_random_field(nx: int, ny: int, nz: int, amplitude: float, seed: int,
                        k_max: int = 3):
    """Seeded smooth random vector field [3][N]: a sum of low-wavenumber
    Fourier modes, scaled to max |component| = amplitude."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = grid_coords(nx, ny, nz)
    out = np.zeros((3, x.size))
    for a in range(3):
        for _ in range(6):
            k = rng.integers(0, k_max + 1, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            c = rng.normal()
            out[a] += c * np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
    m = np.abs(out).max()
    return out * (amplitude / m if m > 0 else 0.0)
