"""Torch-owned device buffers for one level, driven through the C ABI.

PyTorch provides device memory and the stream; every computation happens in
libcslbm.so.  A ``Level`` owns two population buffers (current and next), an
optional scalar pair, optional cell flags and an optional body-force field.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi

F32, F16S = _capi.F32, _capi.F16S


@dataclass
class Params:
    """Model parameters of a level (lattice units); defaults are the
    appendix artificial viscosities and the adaptive-relaxation constants."""
    nu: float = 1e-4
    nu_hi: tuple = (0.005, 0.007, 0.009, 0.01)
    a: float = -4.0
    b: float = 5.0
    g_max: float = 0.1
    adaptive: bool = True
    tau_s: float = 0.51
    beta: float = 0.0
    s_ref: float = 0.0
    u_in: tuple = (0.0, 0.0, 0.0)
    s_in: float = 0.0
    grad_mode: int = 0     # 0: local strain-rate estimate; 1: |grad u|_F by differences
    gmax_running: bool = False   # grad_mode 1: g_max = the field's maximum gradient

    def to_c(self) -> _capi.CslbmParams:
        return _capi.CslbmParams(
            self.nu, (C.c_double * 4)(*self.nu_hi), self.a, self.b, self.g_max,
            int(self.adaptive), int(self.grad_mode), int(self.gmax_running), self.tau_s,
            self.beta, self.s_ref, (C.c_double * 3)(*self.u_in), self.s_in)


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous()
    return t.data_ptr()


def brick_layout(mask: np.ndarray, nx: int, ny: int, nz: int):
    """Storage layout of the stored bricks ``mask`` (bool [nz/8][ny/8][nx/8])
    of an nx*ny*nz box: the brick table (index of each brick among the
    stored ones, -1 for the others, x fastest), the stored bricks'
    coordinates [n_bricks * 3] and, for every storage index (512 per brick,
    x fastest inside the brick), the cell's index in the box."""
    mask = np.asarray(mask, bool)
    bnx, bny, bnz = nx // 8, ny // 8, nz // 8
    if (nx % 8 or ny % 8 or nz % 8) or mask.shape != (bnz, bny, bnx):
        raise ValueError(f"brick mask {mask.shape} does not tile the box {nx}x{ny}x{nz} with 8x8x8 bricks")
    ids = np.flatnonzero(mask.reshape(-1))
    if ids.size == 0:
        raise ValueError("no stored brick")
    table = np.full(mask.size, -1, np.int32)
    table[ids] = np.arange(ids.size, dtype=np.int32)
    bx, by, bz = ids % bnx, (ids // bnx) % bny, ids // (bnx * bny)
    origin = np.stack([bx, by, bz], axis=1).astype(np.int32).reshape(-1)
    l = np.arange(512)
    lx, ly, lz = l % 8, (l // 8) % 8, l // 64
    X = (bx[:, None] * 8 + lx[None, :]).reshape(-1)
    Y = (by[:, None] * 8 + ly[None, :]).reshape(-1)
    Z = (bz[:, None] * 8 + lz[None, :]).reshape(-1)
    return table, origin, (X + nx * (Y + ny * Z)).astype(np.int64)


class Level:
    """One uniform D3Q27 level of nx*ny*nz cells on the current CUDA device.

    With ``bricks`` (a boolean mask over the 8x8x8 bricks of the box, shape
    (nz/8, ny/8, nx/8)) only the marked bricks are stored: ``n`` is then the
    number of stored cells, every per-cell array of the level (states, flags,
    inputs and outputs of the calls) is in storage order, and ``flags`` /
    ``force`` may be given over the whole box (they are gathered).
    ``dense_index`` maps storage order to box order."""

    def __init__(self, nx: int, ny: int, nz: int, params: Params | None = None, *,
                 storage: int = F32, scalar: bool = False, periodic: int = 7,
                 flags: np.ndarray | torch.Tensor | None = None,
                 force: np.ndarray | torch.Tensor | None = None,
                 origin=(0.0, 0.0, 0.0), dx: float = 1.0, device=None, bricks=None):
        lib = _capi.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n_box = self.nx * self.ny * self.nz
        self.n = self.n_box
        self.params = params or Params()
        self.storage = storage
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.brick_table = self.brick_origin = None
        self.n_bricks = 0
        self.dense_index = None
        if bricks is not None:
            self._init_bricks(np.asarray(bricks, dtype=bool))
            periodic = 0
            if flags is not None and np.asarray(flags).size == self.n_box:
                flags = np.asarray(flags, dtype=np.uint8).reshape(-1)[self.dense_index]
            if force is not None:
                raise ValueError("brick levels take no force field")
        plane = lib.cslbm_plane_stride(self.nx, self.ny, self.nz) if bricks is None else \
            lib.cslbm_plane_stride(self.n, 1, 1)
        if plane < 0:
            raise _capi.CslbmError(plane, "cslbm_plane_stride", lib.cslbm_last_error().decode())
        self.plane = int(plane)
        dt = torch.float32 if storage == F32 else torch.float16
        self.f = torch.zeros(27 * self.plane, dtype=dt, device=self.device)
        self.f_next = torch.zeros_like(self.f)
        self.g = self.g_next = None
        if scalar:
            self.g = torch.zeros(7 * self.plane, dtype=torch.float32, device=self.device)
            self.g_next = torch.zeros_like(self.g)
        self.flags = None
        self.links = None
        self.wall_cells = 0
        if flags is not None:
            fl = torch.as_tensor(np.asarray(flags, dtype=np.uint8) if not torch.is_tensor(flags)
                                 else flags).to(self.device, torch.uint8).reshape(-1)
            assert fl.numel() == self.n
            self.wall_cells = int(((fl & 7) == _capi.WALL).sum())
            self.flags = torch.zeros(self.plane, dtype=torch.uint8, device=self.device)
            self.flags[: self.n] = fl
            self.links = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.force = None
        if force is not None:
            ft = torch.as_tensor(np.asarray(force) if not torch.is_tensor(force) else force)
            ft = ft.to(self.device, torch.float32).reshape(3, self.n)
            self.force = torch.zeros(3, self.plane, dtype=torch.float32, device=self.device)
            self.force[:, : self.n] = ft
            self.force = self.force.reshape(-1)
        self.vel = self.vel_next = self.gmax_buf = None
        if self.params.grad_mode == 1:
            self.vel = torch.zeros(3 * self.n, dtype=torch.float32, device=self.device)
            self.vel_next = torch.zeros_like(self.vel)
            self.gmax_buf = torch.zeros(_capi.GMAX_BUF, dtype=torch.float32, device=self.device)
        self.c = _capi.CslbmLevel()
        self.c.nx, self.c.ny, self.c.nz = self.nx, self.ny, self.nz
        self.c.storage = storage
        self.c.periodic = periodic
        self.c.plane = self.plane
        self.c.origin = (C.c_double * 3)(*origin)
        self.c.dx = dx
        self._sync_struct()
        if self.flags is not None:
            _capi.call("cslbm_prepare_flags", C.byref(self.c), _stream_handle())

    def _init_bricks(self, mask: np.ndarray):
        table, origin, self.dense_index = brick_layout(mask, self.nx, self.ny, self.nz)
        self.n_bricks = origin.size // 3
        self.n = self.n_bricks * 512
        self._table = table
        self.brick_table = torch.as_tensor(table, device=self.device)
        self.brick_origin = torch.as_tensor(origin, device=self.device)

    def storage_of(self, dense: np.ndarray) -> np.ndarray:
        """Storage indices of box cells (box order for a dense level; -1 for
        cells of a brick level that are not stored)."""
        dense = np.asarray(dense, dtype=np.int64)
        if self.dense_index is None:
            return dense
        # through the brick table: 512 * brick + lx + 8 ly + 64 lz, on the
        # level's device when it has one (the lists run to millions of cells)
        nx, ny, bnx, bny = self.nx, self.ny, self.nx // 8, self.ny // 8
        if dense.size and (dense.min() < 0 or dense.max() >= nx * ny * self.nz):
            raise ValueError("box cell index outside the level's box")
        table = getattr(self, "brick_table", None)
        if table is not None and table.is_cuda:
            d = torch.as_tensor(dense, device=table.device)
            x, y, z = d % nx, (d // nx) % ny, d // (nx * ny)
            b = table[(x >> 3) + bnx * ((y >> 3) + bny * (z >> 3))].to(torch.int64)
            return torch.where(b < 0, -1, b * 512 + (x & 7) + 8 * (y & 7) + 64 * (z & 7)).cpu().numpy()
        x, y, z = dense % nx, (dense // nx) % ny, dense // (nx * ny)
        b = self._table[(x >> 3) + bnx * ((y >> 3) + bny * (z >> 3))].astype(np.int64)
        return np.where(b < 0, -1, b * 512 + (x & 7) + 8 * (y & 7) + 64 * (z & 7))

    def to_storage(self, box_values: np.ndarray) -> np.ndarray:
        """Per-cell values over the box ([..., n_box]) in storage order."""
        v = np.asarray(box_values)
        return v if self.dense_index is None else v[..., self.dense_index]

    # -- struct <-> tensors ------------------------------------------------
    def _sync_struct(self):
        self.c.f = _dev_ptr(self.f)
        self.c.f_next = _dev_ptr(self.f_next)
        self.c.g = _dev_ptr(self.g)
        self.c.g_next = _dev_ptr(self.g_next)
        self.c.flags = _dev_ptr(self.flags)
        self.c.links = _dev_ptr(self.links)
        self.c.force = _dev_ptr(self.force)
        self.c.vel = _dev_ptr(self.vel)
        self.c.vel_next = _dev_ptr(self.vel_next)
        self.c.gmax_buf = _dev_ptr(self.gmax_buf)
        self.c.brick_table = _dev_ptr(self.brick_table)
        self.c.brick_origin = _dev_ptr(self.brick_origin)
        self.c.n_bricks = self.n_bricks
        self.c.wall_cells = self.wall_cells
        self.c.p = self.params.to_c()

    def set_params(self, params: Params):
        self.params = params
        self.c.p = params.to_c()
        if params.grad_mode == 1 and self.vel is None:
            # the velocity of the current state, as the gradient mode needs it
            self.vel = torch.zeros(3 * self.n, dtype=torch.float32, device=self.device)
            self.vel_next = torch.zeros_like(self.vel)
            self.gmax_buf = torch.zeros(_capi.GMAX_BUF, dtype=torch.float32, device=self.device)
            self._sync_struct()
            _capi.call("cslbm_read_macro", C.byref(self.c), None, _dev_ptr(self.vel), None,
                       _stream_handle())

    def set_flags(self, flags):
        flags = np.asarray(flags, dtype=np.uint8).reshape(-1)
        if self.dense_index is not None and flags.size == self.n_box:
            flags = flags[self.dense_index]
        fl = torch.as_tensor(flags).to(self.device).reshape(-1)
        if self.flags is None:
            self.flags = torch.zeros(self.plane, dtype=torch.uint8, device=self.device)
            self.links = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.flags[: self.n] = fl
        self.wall_cells = int(np.count_nonzero((flags & 7) == _capi.WALL))
        self._sync_struct()
        _capi.call("cslbm_prepare_flags", C.byref(self.c), _stream_handle())

    # -- C-ABI calls ---------------------------------------------------------
    def init_equilibrium(self, rho=None, u=None, s=None, stream=None):
        dev = self.device
        u_t = torch.as_tensor(np.asarray(u, dtype=np.float32)).to(dev).reshape(3, self.n).contiguous()
        r_t = None if rho is None else torch.as_tensor(np.asarray(rho, dtype=np.float32)).to(dev).reshape(-1).contiguous()
        s_t = None if s is None else torch.as_tensor(np.asarray(s, dtype=np.float32)).to(dev).reshape(-1).contiguous()
        self._sync_struct()
        _capi.call("cslbm_init_equilibrium", C.byref(self.c), _dev_ptr(r_t), _dev_ptr(u_t),
                   _dev_ptr(s_t), _stream_handle(stream))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def set_populations(self, f, g=None, shifted: bool = False, stream=None):
        dev = self.device
        f_t = torch.as_tensor(np.asarray(f, dtype=np.float32) if not torch.is_tensor(f) else f)
        f_t = f_t.to(dev, torch.float32).reshape(27, self.n).contiguous()
        g_t = None
        if g is not None:
            g_t = torch.as_tensor(np.asarray(g, dtype=np.float32) if not torch.is_tensor(g) else g)
            g_t = g_t.to(dev, torch.float32).reshape(7, self.n).contiguous()
        self._sync_struct()
        _capi.call("cslbm_set_populations", C.byref(self.c), _dev_ptr(f_t), _dev_ptr(g_t),
                   int(shifted), _stream_handle(stream))
        torch.cuda.synchronize()

    def get_populations(self, shifted: bool = False, stream=None):
        out = torch.empty(27, self.n, dtype=torch.float32, device=self.device)
        gout = None if self.g is None else torch.empty(7, self.n, dtype=torch.float32, device=self.device)
        self._sync_struct()
        _capi.call("cslbm_get_populations", C.byref(self.c), _dev_ptr(out), _dev_ptr(gout),
                   int(shifted), _stream_handle(stream))
        return out, gout

    def step(self, n_steps: int = 1, stream=None):
        self._sync_struct()
        _capi.call("cslbm_step", C.byref(self.c), int(n_steps), _stream_handle(stream))
        if n_steps % 2:
            self.f, self.f_next = self.f_next, self.f
            if self.g is not None:
                self.g, self.g_next = self.g_next, self.g
            if self.vel is not None:
                self.vel, self.vel_next = self.vel_next, self.vel
        assert self.c.f == self.f.data_ptr()

    def read_macro(self, stream=None):
        rho = torch.empty(self.n, dtype=torch.float32, device=self.device)
        u = torch.empty(3, self.n, dtype=torch.float32, device=self.device)
        s = None if self.g is None else torch.empty(self.n, dtype=torch.float32, device=self.device)
        self._sync_struct()
        _capi.call("cslbm_read_macro", C.byref(self.c), _dev_ptr(rho), _dev_ptr(u), _dev_ptr(s),
                   _stream_handle(stream))
        return rho, u, s

    def vorticity(self, stream=None):
        """(|curl u|, |u|) of the stored state, dense [N] each."""
        out = torch.empty(self.n, dtype=torch.float32, device=self.device)
        speed = torch.empty(self.n, dtype=torch.float32, device=self.device)
        self._sync_struct()
        _capi.call("cslbm_vorticity", C.byref(self.c), _dev_ptr(out), _dev_ptr(speed),
                   _stream_handle(stream))
        return out, speed

    def conserved(self, stream=None) -> np.ndarray:
        out = (C.c_double * 5)()
        self._sync_struct()
        _capi.call("cslbm_conserved_f64", C.byref(self.c), out, _stream_handle(stream))
        return np.array(out[:])

    def count_nonfinite(self, stream=None) -> int:
        n = C.c_int64(0)
        self._sync_struct()
        lib = _capi.load()
        rc = lib.cslbm_check_finite(C.byref(self.c), C.byref(n), _stream_handle(stream))
        if rc not in (_capi.OK, _capi.ERR_NONFINITE):
            raise _capi.CslbmError(rc, "cslbm_check_finite", lib.cslbm_last_error().decode())
        return int(n.value)

    # -- differentiation support ---------------------------------------------
    def _struct_with_state(self, f: torch.Tensor, g: torch.Tensor | None) -> _capi.CslbmLevel:
        self._sync_struct()
        c = _capi.CslbmLevel()
        C.pointer(c)[0] = self.c
        c.f = _dev_ptr(f)
        c.g = _dev_ptr(g)
        return c

    def step_store(self, f_start, g_start, f_states, g_states, stream=None):
        """len(f_states) steps from (f_start, g_start), writing every state."""
        n = len(f_states)
        c = self._struct_with_state(f_start, g_start)
        fp = (C.c_void_p * max(n, 1))(*[t.data_ptr() for t in f_states])
        gp = None
        if g_start is not None:
            gp = (C.c_void_p * max(n, 1))(*[t.data_ptr() for t in g_states])
        _capi.call("cslbm_step_store", C.byref(c), n, fp, gp, _stream_handle(stream))

    def adjoint_step(self, f_state, g_state, lam_next, mu_next, lam, mu, dtheta, stream=None):
        """lam = dL/df(n) from lam_next = dL/df(n+1) for the step that read
        (f_state, g_state); dtheta accumulates dL/dtheta."""
        c = self._struct_with_state(f_state, g_state)
        _capi.call("cslbm_adjoint_step", C.byref(c), _dev_ptr(lam_next), _dev_ptr(mu_next),
                   _dev_ptr(lam), _dev_ptr(mu), _dev_ptr(dtheta), _stream_handle(stream))
