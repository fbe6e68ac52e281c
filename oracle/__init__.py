"""Plain FP64 CPU oracle of the central-moment lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It wraps ``libcmr_oracle.so``
(built from ``cmr_oracle.c`` with gcc) through ctypes and shares nothing with
the GPU library.  All arrays are float64 numpy arrays in the layout documented
in ``cmr_oracle.h``: populations ``[27][N]`` with ``N = nx*ny*nz``, x fastest.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cmr_oracle.c")
LIB = os.path.join(HERE, "libcmr_oracle.so")

FLUID, SOLID, INLET, OUTFLOW, GHOST, NEUMANN, WALL = 0, 1, 2, 3, 4, 5, 6

_dp = C.POINTER(C.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over cells)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nu", C.c_double), ("nu_hi", C.c_double * 4), ("a", C.c_double),
                ("b", C.c_double), ("g_max", C.c_double), ("adaptive", C.c_int32),
                ("grad_mode", C.c_int32), ("tau_s", C.c_double), ("beta", C.c_double),
                ("s_ref", C.c_double)]


class _Domain(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32), ("flags", C.POINTER(C.c_uint8)),
                ("theta", _dp), ("u_in", C.c_double * 3), ("s_in", C.c_double)]


class _Scale(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("periodic", C.c_int32),
                ("origin", C.c_double * 3), ("dx", C.c_double), ("nu", C.c_double),
                ("tau_s", C.c_double)]


@dataclass
class Params:
    """Relaxation parameters (appendix values by default)."""
    nu: float = 1e-4
    nu_hi: tuple = (0.005, 0.007, 0.009, 0.01)
    a: float = -4.0
    b: float = 5.0
    g_max: float = 0.1
    adaptive: bool = True
    tau_s: float = 0.51
    beta: float = 0.0
    s_ref: float = 0.0
    grad_mode: int = 0          # 0: local strain-rate estimate; 1: |grad u|_F by differences
    gmax_running: bool = False  # grad_mode 1: g_max of each step = max of its gradient field

    def c(self) -> _Params:
        return _Params(self.nu, (C.c_double * 4)(*self.nu_hi), self.a, self.b,
                       self.g_max, int(self.adaptive), int(self.grad_mode), self.tau_s, self.beta,
                       self.s_ref)


@dataclass
class Domain:
    nx: int
    ny: int
    nz: int
    periodic: int = 7
    flags: np.ndarray | None = None      # uint8 [N]
    theta: np.ndarray | None = None      # float64 [3][N]
    u_in: tuple = (0.0, 0.0, 0.0)
    s_in: float = 0.0
    _keep: list = field(default_factory=list, repr=False)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def c(self) -> _Domain:
        self._keep = []
        fl = None
        if self.flags is not None:
            a = np.ascontiguousarray(self.flags, dtype=np.uint8).reshape(-1)
            assert a.size == self.n
            self._keep.append(a)
            fl = a.ctypes.data_as(C.POINTER(C.c_uint8))
        th = None
        if self.theta is not None:
            t = np.ascontiguousarray(self.theta, dtype=np.float64).reshape(-1)
            assert t.size == 3 * self.n
            self._keep.append(t)
            th = t.ctypes.data_as(_dp)
        return _Domain(self.nx, self.ny, self.nz, self.periodic, fl, th,
                       (C.c_double * 3)(*self.u_in), self.s_in)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.oracle_velocities.argtypes = [C.POINTER(C.c_int32)]
        L.oracle_weights.argtypes = [_dp]
        L.oracle_basis.argtypes = [_dp, _dp]
        L.oracle_meq.argtypes = [C.c_double, _dp, _dp]
        L.oracle_collide.argtypes = [_dp, _dp, C.POINTER(_Params), _dp, _dp, _dp]
        L.oracle_equilibrium.argtypes = [C.c_double, _dp, _dp]
        L.oracle_init.argtypes = [C.POINTER(_Domain), _dp, _dp, _dp, _dp, _dp]
        L.oracle_step.argtypes = [C.POINTER(_Domain), C.POINTER(_Params), _dp, _dp, _dp, _dp]
        L.oracle_stream.argtypes = [C.POINTER(_Domain), _dp, _dp, _dp, _dp]
        L.oracle_step_cells.argtypes = [C.POINTER(_Domain), C.POINTER(_Params), _dp, _dp,
                                        C.POINTER(C.c_int64), C.c_int64, _dp, _dp]
        L.oracle_macro.argtypes = [C.POINTER(_Domain), C.POINTER(_Params), _dp, _dp, _dp, _dp, _dp]
        L.oracle_grad_field.argtypes = [C.POINTER(_Domain), C.POINTER(_Params), _dp, _dp, _dp]
        L.oracle_collide_g.argtypes = [_dp, _dp, C.POINTER(_Params), C.c_double, _dp, _dp]
        L.oracle_exchange.argtypes = [C.POINTER(_Scale), _dp, _dp, _dp, _dp, C.c_double,
                                      C.POINTER(_Scale), C.POINTER(C.c_int64), C.c_int64, _dp, _dp]
        L.oracle_wall_regularize.argtypes = [_dp, C.POINTER(C.c_int32), _dp, _dp]
        L.oracle_time_interp.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_int64, _dp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def velocities() -> np.ndarray:
    c = np.zeros(81, dtype=np.int32)
    lib().oracle_velocities(c.ctypes.data_as(C.POINTER(C.c_int32)))
    return c.reshape(27, 3)


def weights() -> np.ndarray:
    w = np.zeros(27)
    lib().oracle_weights(_p(w))
    return w


def basis(u) -> np.ndarray:
    u = _f64(u, 3)
    M = np.zeros(729)
    lib().oracle_basis(_p(u), _p(M))
    return M.reshape(27, 27)


def meq(rho, u) -> np.ndarray:
    u = _f64(u, 3)
    m = np.zeros(27)
    lib().oracle_meq(float(rho), _p(u), _p(m))
    return m


def collide(f, params: Params, F=None, S_override=None):
    """One-cell collision; returns (f_post[27], diag dict)."""
    f = _f64(f, 27)
    F = None if F is None else _f64(F, 3)
    S = None if S_override is None else _f64(S_override, 27)
    out = np.zeros(27)
    diag = np.zeros(6)
    pc = params.c()
    rc = lib().oracle_collide(_p(f), _p(F), C.byref(pc), _p(S), _p(out), _p(diag))
    if rc != 0:
        raise RuntimeError("oracle_collide failed")
    return out, dict(zip(("rho", "ux", "uy", "uz", "G", "phi"), diag))


def equilibrium(rho, u) -> np.ndarray:
    u = _f64(u, 3)
    f = np.zeros(27)
    if lib().oracle_equilibrium(float(rho), _p(u), _p(f)) != 0:
        raise RuntimeError("oracle_equilibrium failed")
    return f


def init(dom: Domain, rho, u, s=None, with_scalar=False):
    n = dom.n
    rho = _f64(rho, n)
    u = _f64(u, 3 * n)
    s = None if s is None else _f64(s, n)
    f = np.zeros((27, n))
    g = np.zeros((7, n)) if (with_scalar or s is not None) else None
    dc = dom.c()
    if lib().oracle_init(C.byref(dc), _p(rho), _p(u), _p(s), _p(f), _p(g)) != 0:
        raise RuntimeError("oracle_init failed")
    return f, g


def step(dom: Domain, params: Params, f, g=None, n_steps: int = 1):
    n = dom.n
    f = _f64(f, 27 * n).reshape(27, n).copy()
    g = None if g is None else _f64(g, 7 * n).reshape(7, n).copy()
    fo = np.empty_like(f)
    go = None if g is None else np.empty_like(g)
    dc, pc = dom.c(), params.c()
    for _ in range(n_steps):
        if params.gmax_running and params.grad_mode == 1:
            # section "Adaptive relaxation": g_max normalises by the maximum
            # gradient magnitude, here the maximum of this step's field
            gm = float(np.max(grad_field(dom, params, f, g)))
            pc.g_max = gm if gm > 0.0 else 1.0
        if lib().oracle_step(C.byref(dc), C.byref(pc), _p(f), _p(g), _p(fo), _p(go)) != 0:
            raise RuntimeError("oracle_step failed")
        f, fo = fo, f
        if g is not None:
            g, go = go, g
    return f, g


def stream(dom: Domain, f, g=None):
    """Pull streaming alone (fluid cells gather, other cells copy)."""
    n = dom.n
    f = _f64(f, 27 * n)
    g = None if g is None else _f64(g, 7 * n)
    fo = np.zeros((27, n))
    go = None if g is None else np.zeros((7, n))
    dc = dom.c()
    lib().oracle_stream(C.byref(dc), _p(f), _p(g), _p(fo), _p(go))
    return fo, go


def step_cells(dom: Domain, params: Params, f, cells, g=None):
    n = dom.n
    f = _f64(f, 27 * n)
    g = None if g is None else _f64(g, 7 * n)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    k = cells.size
    fo = np.zeros((27, k))
    go = None if g is None else np.zeros((7, k))
    dc, pc = dom.c(), params.c()
    rc = lib().oracle_step_cells(C.byref(dc), C.byref(pc), _p(f), _p(g),
                                 cells.ctypes.data_as(C.POINTER(C.c_int64)), k, _p(fo), _p(go))
    if rc != 0:
        raise RuntimeError("oracle_step_cells failed")
    return fo, go


def macro(dom: Domain, params: Params, f, g=None):
    n = dom.n
    f = _f64(f, 27 * n)
    g = None if g is None else _f64(g, 7 * n)
    rho = np.zeros(n)
    u = np.zeros((3, n))
    s = np.zeros(n) if g is not None else None
    dc, pc = dom.c(), params.c()
    lib().oracle_macro(C.byref(dc), C.byref(pc), _p(f), _p(g), _p(rho), _p(u), _p(s))
    return rho, u, s


def grad_field(dom: Domain, params: Params, f, g=None):
    """|grad u|_F of the read-back velocity of the state (f, g) [N]."""
    n = dom.n
    f = _f64(f, 27 * n)
    g = None if g is None else _f64(g, 7 * n)
    G = np.zeros(n)
    dc, pc = dom.c(), params.c()
    if lib().oracle_grad_field(C.byref(dc), C.byref(pc), _p(f), _p(g), _p(G)) != 0:
        raise RuntimeError("oracle_grad_field failed")
    return G


def collide_g(f, params: Params, G: float, F=None):
    """One cell's collision with the adaptive factor's G given."""
    f = _f64(f, 27)
    Fv = np.zeros(3) if F is None else _f64(F, 3)
    out = np.zeros(27)
    diag = np.zeros(6)
    pc = params.c()
    if lib().oracle_collide_g(_p(f), _p(Fv), C.byref(pc), float(G), _p(out), _p(diag)) != 0:
        raise RuntimeError("oracle_collide_g failed")
    return out, dict(zip(("rho", "ux", "uy", "uz", "G", "phi"), diag))


def _scale_c(nx, ny, nz, periodic, origin, dx, nu, tau_s=0.0) -> _Scale:
    return _Scale(nx, ny, nz, periodic, (C.c_double * 3)(*origin), dx, nu, tau_s)


def exchange(src: dict, fA, fB, w, dst: dict, cells, f_out, gA=None, gB=None, g_out=None):
    """Map source-scale states (time weight w between fA and fB) onto the
    listed cells of the destination scale; writes f_out (and g_out) in place.
    src/dst: dicts with nx, ny, nz, periodic, origin, dx, nu, tau_s."""
    ns = src["nx"] * src["ny"] * src["nz"]
    nd = dst["nx"] * dst["ny"] * dst["nz"]
    fA = _f64(fA, 27 * ns)
    fB = _f64(fB, 27 * ns)
    gA = None if gA is None else _f64(gA, 7 * ns)
    gB = None if gB is None else _f64(gB, 7 * ns)
    assert f_out.dtype == np.float64 and f_out.flags.c_contiguous and f_out.size == 27 * nd
    if g_out is not None:
        assert g_out.dtype == np.float64 and g_out.flags.c_contiguous and g_out.size == 7 * nd
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    sc = _scale_c(src["nx"], src["ny"], src["nz"], src["periodic"], src["origin"], src["dx"],
                  src["nu"], src.get("tau_s", 0.0))
    dc = _scale_c(dst["nx"], dst["ny"], dst["nz"], dst["periodic"], dst["origin"], dst["dx"],
                  dst["nu"], dst.get("tau_s", 0.0))
    rc = lib().oracle_exchange(C.byref(sc), _p(fA), _p(fB), _p(gA), _p(gB), float(w), C.byref(dc),
                               cells.ctypes.data_as(C.POINTER(C.c_int64)), cells.size,
                               _p(f_out), _p(g_out))
    if rc != 0:
        raise RuntimeError("oracle_exchange failed (stencil outside the source box?)")


def wall_regularize(f, n, F=None):
    """Regularized no-slip wall node (kind WALL) applied to one cell's
    pulled populations f[27]; n: wall normal (unit axis vector into the
    wall), F: body force at the node."""
    f = _f64(f, 27)
    nn = np.ascontiguousarray(n, dtype=np.int32)
    assert nn.size == 3
    Fv = None if F is None else _f64(F, 3)
    out = np.zeros(27)
    if lib().oracle_wall_regularize(_p(f), nn.ctypes.data_as(C.POINTER(C.c_int32)), _p(Fv),
                                    _p(out)) != 0:
        raise ValueError("bad wall normal")
    return out


def time_interp(s0, s1, s2, t, t_eval):
    s0 = _f64(s0)
    s1 = _f64(s1, s0.size)
    s2 = _f64(s2, s0.size)
    out = np.empty_like(s0)
    lib().oracle_time_interp(_p(s0), _p(s1), _p(s2), float(t[0]), float(t[1]), float(t[2]),
                             float(t_eval), s0.size, _p(out))
    return out
