"""Plain multi-scale scheduler of the oracle (Algorithm 1 and the sections
"Temporal alignment and scale mapping" and "Handling multiple scales").

TEST INFRASTRUCTURE ONLY.  Written independently of the GPU driver: it calls
the oracle's step, exchange and time-interpolation functions in the order of
Algorithm 1, with the readings listed below.

Readings (each also listed in the design doc):
  * scale 0 is the reference scale s0 and covers the whole domain; every
    other scale is a box of lattice points origin + (x, y, z) dx nested in
    its parent, the nearest coarser scale (scale i - 1);
  * the boundary of a finer scale is its one-cell outer shell (GHOST cells):
    never collided, written only by prior-mapping;
  * alpha_i = dx_0 / dx_i; the scale's viscosity is alpha_i nu_0 (invariant
    local Reynolds number, eq. S_relation); l = floor(alpha_i) + 1 sub-steps;
  * before each of the first l - 1 sub-steps the shell is prior-mapped from
    the parent blended in time between its states at t_n and t_n + dt_0;
    the paper names the two end points but not the time, and the reading
    here is the sub-step's start time, weight (k - 1) / alpha_i for
    sub-step k (the pull reads the shell at the start of the sub-step);
  * before the final sub-step (k = l) the shell is mapped directly from the
    parent at t_n + dt_0 (weight 1), as section "Temporal alignment and
    scale mapping" states;
  * after the sub-steps the whole scale is interpolated in time by the
    quadratic through t = 0, (l - 1)/alpha_i, l/alpha_i evaluated at 1, and
    the shell is mapped again from the parent at t_n + dt_0;
  * post-mapping writes every larger scale (spacing above the scale's own,
    far-field scales included) at its FLUID cells whose trilinear stencil
    in scale i consists of FLUID cells of scale i; finer scales run and
    post-map in index order.

Far-field scales (spacing larger than the reference scale, alpha_c < 1)
follow the reversed rules of section "Handling multiple scales": the region
they share with their parent is GHOST in their flags and is mapped from the
parent in full (at t_n before their step and again at t_n + dt_0 after it);
they take one step and interpolate linearly back to t_n + dt_0; they
post-map only onto the parent's ghost shell; their own outer faces are
Neumann cells.  As in Algorithm 1 they advance together with the reference
scale, before the loop over finer scales.  Their shared region is GHOST,
so a finer scale (which lies inside the reference window) finds no FLUID
target in them unless an object is resolved differently on the two scales.

Pins (CPU tests): a finer scale with the reference spacing on coincident
points reproduces the single-scale run (integer alpha, mapping = identity);
uniform flow stays uniform on three nested scales at alpha 1.5 and 2; a
two-scale Taylor-Green vortex (alpha = 1.5) keeps the closed-form decay
within 2 %; under a uniform body force (momentum linear in time in closed
form) the shell before every sub-step holds the parent's state at the time
the schedule names, at alpha 1.5, 2 and 2.5.  The start-time reading of the
first l - 1 weights and the shell and post-region rules are readings: their
parity is pinned only by those checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import FLUID, GHOST, SOLID, Domain, Params, exchange, step, time_interp


@dataclass
class OScale:
    nx: int
    ny: int
    nz: int
    dx: float
    origin: tuple
    params: Params               # nu already in this scale's lattice units
    flags: np.ndarray            # uint8 [N]; finer scales carry a GHOST shell
    periodic: int = 0
    parent: int = -1
    u_in: tuple = (0.0, 0.0, 0.0)
    s_in: float = 0.0
    f: np.ndarray | None = None  # [27][N] state at the current reference time
    g: np.ndarray | None = None  # [7][N] or None
    ghosts: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    post: dict = field(default_factory=dict)   # coarser scale index -> cells of that scale
    theta: np.ndarray | None = None             # [3][N] body force, lattice units of this scale

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def domain(self) -> Domain:
        return Domain(self.nx, self.ny, self.nz, periodic=self.periodic, flags=self.flags,
                      theta=self.theta, u_in=self.u_in, s_in=self.s_in)

    def geom(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, periodic=self.periodic,
                    origin=tuple(self.origin), dx=self.dx, nu=self.params.nu,
                    tau_s=self.params.tau_s if self.g is not None else 0.0)

    def positions(self):
        z, y, x = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx),
                              indexing="ij")
        return (self.origin[0] + x.reshape(-1) * self.dx, self.origin[1] + y.reshape(-1) * self.dx,
                self.origin[2] + z.reshape(-1) * self.dx)


def shell_ghosts(s: OScale) -> np.ndarray:
    return np.flatnonzero(s.flags == GHOST).astype(np.int64)


def post_targets(coarse: OScale, fine: OScale) -> np.ndarray:
    """Cells of `coarse` to be overwritten from `fine`: FLUID cells whose
    trilinear stencil in `fine` (corners with non-zero weight) lies inside
    the fine box and consists of FLUID cells."""
    px, py, pz = coarse.positions()
    out = []
    for c in np.flatnonzero(coarse.flags == FLUID):
        p = (px[c], py[c], pz[c])
        ok = True
        base, frac = [], []
        for a, n in enumerate((fine.nx, fine.ny, fine.nz)):
            q = (p[a] - fine.origin[a]) / fine.dx
            b = math.floor(q)
            base.append(b)
            frac.append(q - b)
        for corner in range(8):
            o = (corner & 1, (corner >> 1) & 1, (corner >> 2) & 1)
            wt = 1.0
            for a in range(3):
                wt *= frac[a] if o[a] else 1.0 - frac[a]
            if wt == 0.0:
                continue
            idx = [base[a] + o[a] for a in range(3)]
            if not (0 <= idx[0] < fine.nx and 0 <= idx[1] < fine.ny and 0 <= idx[2] < fine.nz):
                ok = False
                break
            fc = idx[0] + fine.nx * (idx[1] + fine.ny * idx[2])
            if fine.flags[fc] != FLUID:
                ok = False
                break
        if ok:
            out.append(c)
    return np.array(out, dtype=np.int64)


def is_coarse(scales: list[OScale], i: int) -> bool:
    """A scale with a larger spacing than the reference scale (far field)."""
    return i > 0 and scales[i].dx > scales[0].dx


def prepare(scales: list[OScale]):
    """Fill the ghost and post-mapping lists of every scale but the reference.

    A finer scale's ghosts are its one-cell shell; it post-maps onto every
    larger scale: the scales before it (its parent chain) and the far-field
    scales.  A coarser (far-field) scale is the reverse
    (section "Handling multiple scales"): its ghosts are the whole region it
    shares with its parent (the finer scale it surrounds), marked GHOST by
    the caller, and it post-maps only onto the parent's ghost shell."""
    for i, s in enumerate(scales):
        if i == 0:
            continue
        if is_coarse(scales, i):
            s.ghosts = np.flatnonzero(s.flags == GHOST).astype(np.int64)
            s.post = {s.parent: shell_ghosts(scales[s.parent])}
        else:
            s.ghosts = shell_ghosts(s)
            s.post = {j: post_targets(scales[j], s) for j in range(len(scales))
                      if j < i or is_coarse(scales, j)}


def multiscale_step(scales: list[OScale], n_ref: int = 1):
    """Advance every scale by n_ref reference steps (Algorithm 1)."""
    for _ in range(n_ref):
        # the reference scale and the far-field scales take their step
        # (first statement of Algorithm 1's loop)
        s0 = scales[0]
        A0, gA0 = s0.f, s0.g
        B0, gB0 = step(s0.domain(), s0.params, s0.f, s0.g)
        states = {0: (A0, B0, gA0, gB0)}
        # far-field scales (section "Temporal alignment and scale mapping"):
        # the shared region is mapped from the parent at t_n, one step of
        # dt_c = dt_0 / alpha_c, linear interpolation back to t_n + dt_0, the
        # shared region mapped again at t_n + dt_0, then the parent's
        # boundary shell is mapped from this scale
        for i in range(1, len(scales)):
            if not is_coarse(scales, i):
                continue
            s = scales[i]
            par = scales[s.parent]
            Ap, Bp, gAp, gBp = states[s.parent]
            ac = scales[0].dx / s.dx                     # alpha_c in (0, 1)
            X0 = s.f.copy()
            gX0 = None if s.g is None else s.g.copy()
            exchange(par.geom(), Ap, Bp, 0.0, s.geom(), s.ghosts, X0, gAp, gBp, gX0)
            X1, gX1 = step(s.domain(), s.params, X0, gX0)
            R = (1.0 - ac) * X0 + ac * X1
            gR = None if gX0 is None else (1.0 - ac) * gX0 + ac * gX1
            exchange(par.geom(), Ap, Bp, 1.0, s.geom(), s.ghosts, R, gAp, gBp, gR)
            states[i] = (X0, R, gX0, gR)
            tgt = s.post[s.parent]
            if tgt.size:
                exchange(s.geom(), R, R, 0.0, par.geom(), tgt, Bp, gR, gR, gBp)
        # finer scales, coarse to fine
        for i in range(1, len(scales)):
            if is_coarse(scales, i):
                continue
            s = scales[i]
            par = scales[s.parent]
            Ap, Bp, gAp, gBp = states[s.parent]
            alpha = scales[0].dx / s.dx                  # dx_0 / dx_i
            l = math.floor(alpha) + 1
            X0 = s.f.copy()
            gX0 = None if s.g is None else s.g.copy()
            cur, gcur = X0.copy(), None if gX0 is None else gX0.copy()
            hist = [(X0, gX0)]
            for k in range(1, l + 1):
                # first l - 1 sub-steps: the parent blended at the sub-step's
                # start time; the final one: the parent at t_n + dt_0
                w = 1.0 if k == l else (k - 1) / alpha
                exchange(par.geom(), Ap, Bp, w, s.geom(), s.ghosts, cur, gAp, gBp, gcur)
                if k == 1:
                    X0 = cur.copy()
                    gX0 = None if gcur is None else gcur.copy()
                    hist[0] = (X0, gX0)
                cur, gcur = step(s.domain(), s.params, cur, gcur)
                hist.append((cur, gcur))
            t = (0.0, (l - 1) / alpha, l / alpha)
            R = time_interp(hist[0][0], hist[l - 1][0], hist[l][0], t, 1.0).reshape(27, s.n)
            gR = None
            if s.g is not None:
                gR = time_interp(hist[0][1], hist[l - 1][1], hist[l][1], t, 1.0).reshape(7, s.n)
            exchange(par.geom(), Ap, Bp, 1.0, s.geom(), s.ghosts, R, gAp, gBp, gR)
            states[i] = (X0, R, gX0, gR)
            # post-mapping onto every larger scale, in index order
            for j in sorted(s.post):
                tgt = s.post[j]
                if tgt.size == 0:
                    continue
                Bj, gBj = states[j][1], states[j][3]
                exchange(s.geom(), R, R, 0.0, scales[j].geom(), tgt, Bj, gR, gR, gBj)
        for i, s in enumerate(scales):
            s.f = states[i][1]
            s.g = states[i][3]
    return scales
