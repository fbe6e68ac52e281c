"""Continuous-scale level sets on the GPU (Algorithm 1 through the C ABI).

A ``Hierarchy`` holds a reference ``Level`` (scale 0) and finer levels, each
a box of lattice points ``origin + (x, y, z) * dx`` with a one-cell
``GHOST`` shell, nested in its parent.  It allocates the per-scale work
buffers, builds the prior-mapping (ghost) and post-mapping cell lists, and
calls ``cslbm_multiscale_step``.  All arithmetic runs in libcslbm.so.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch
from scipy import ndimage

from . import _capi
from .level import Level, Params, _stream_handle

FLUID, GHOST = _capi.FLUID, _capi.GHOST


def shell_flags(nx: int, ny: int, nz: int, inner: np.ndarray | None = None) -> np.ndarray:
    """Cell kinds of a finer scale: the one-cell outer shell is GHOST, the
    inside takes `inner` (default FLUID)."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    fl = np.zeros(nx * ny * nz, np.uint8) if inner is None else np.asarray(inner, np.uint8).copy()
    fl[(x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)] = GHOST
    return fl


def _stencil(points: np.ndarray, origin, dx, n):
    """Trilinear stencil of physical points in a lattice: base index and
    fractions per axis (points: [3, K])."""
    q = (points - np.asarray(origin, float)[:, None]) / dx
    base = np.floor(q).astype(np.int64)
    return base, q - base


def _axis_stencil(lo: int, hi: int, c_origin: float, c_dx: float, f_origin: float, f_dx: float):
    """Trilinear stencil along one axis for coarse indices lo..hi: base fine
    index and fraction (the stencil is separable per axis)."""
    q = (c_origin + np.arange(lo, hi + 1) * c_dx - f_origin) / f_dx
    b = np.floor(q)
    return b.astype(np.int64), q - b


def post_cells(coarse_kinds: np.ndarray, coarse_shape, coarse_origin, coarse_dx,
               fine_kinds: np.ndarray, fine_shape, fine_origin, fine_dx) -> np.ndarray:
    """Cells of the coarse scale whose position has a trilinear stencil (the
    corners with non-zero weight) made of FLUID cells inside the fine box.

    The stencil is separable: along each axis a coarse index uses the fine
    index b and, when its fraction is not 0, b + 1.  Staying inside the box
    is a product of per-axis conditions; the corners are then gathered from
    the fine FLUID mask axis by axis (a corner of weight 0 is pointed at b,
    which is checked anyway).  Runs on the GPU when there is one."""
    cnx, cny, cnz = coarse_shape
    fnx, fny, fnz = fine_shape
    fn = (fnx, fny, fnz)
    lo = [max(0, math.floor((fine_origin[a] - coarse_origin[a]) / coarse_dx) - 1) for a in range(3)]
    hi = [min(coarse_shape[a] - 1,
              math.ceil((fine_origin[a] + (fine_shape[a] - 1) * fine_dx - coarse_origin[a]) / coarse_dx) + 1)
          for a in range(3)]
    if any(h < l for l, h in zip(lo, hi)):
        return np.zeros(0, np.int32)
    dev = torch.device("cuda") if torch.cuda.is_available() else torch.device("cpu")
    inside, corner = [], []
    for a in range(3):
        b, t = _axis_stencil(lo[a], hi[a], coarse_origin[a], coarse_dx, fine_origin[a], fine_dx)
        up = t != 0.0                                   # b + 1 has non-zero weight
        inside.append(torch.as_tensor((b >= 0) & (b < fn[a]) & (~up | (b + 1 < fn[a])), device=dev))
        corner.append([torch.as_tensor(np.clip(b + o * up, 0, fn[a] - 1), device=dev) for o in (0, 1)])
    ck = np.asarray(coarse_kinds).reshape(cnz, cny, cnx)[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
    ok = torch.as_tensor(ck == FLUID, device=dev)
    ok &= inside[2][:, None, None] & inside[1][None, :, None] & inside[0][None, None, :]
    fluid = torch.as_tensor(np.asarray(fine_kinds).reshape(fnz, fny, fnx) == FLUID, device=dev)
    for oz in range(2):
        fz = fluid.index_select(0, corner[2][oz])
        for oy in range(2):
            fzy = fz.index_select(1, corner[1][oy])
            for ox in range(2):
                ok &= fzy.index_select(2, corner[0][ox])
    k = torch.nonzero(ok).cpu().numpy()
    if k.size == 0:
        return np.zeros(0, np.int32)
    return ((k[:, 2] + lo[0]) + cnx * ((k[:, 1] + lo[1]) + cny * (k[:, 0] + lo[2]))).astype(np.int32)


def check_prior_stencils(parent_kinds, parent_shape, parent_origin, parent_dx, parent_periodic,
                         fine_shape, fine_origin, fine_dx, ghosts: np.ndarray):
    """Every ghost of a finer scale must interpolate from FLUID cells of its
    parent (inside the box on non-periodic axes).  The stencil is separable:
    per axis and fine index, the parent index of each corner, whether it
    lies inside and whether its weight is non-zero (the product of the
    three axes' weights is non-zero exactly when each is)."""
    g = np.asarray(ghosts, np.int64)
    fnx, fny, _ = fine_shape
    coord = (g % fnx, (g // fnx) % fny, g // (fnx * fny))
    pidx, inside, need = [], [], []
    for a in range(3):
        q = (fine_origin[a] + np.arange(fine_shape[a]) * fine_dx - parent_origin[a]) / parent_dx
        base = np.floor(q)
        t = q - base
        base = base.astype(np.int64)
        per = []
        for o in (0, 1):
            idx = base + o
            if parent_periodic & (1 << a):
                idx %= parent_shape[a]
            ok = (idx >= 0) & (idx < parent_shape[a])
            per.append((np.where(ok, idx, 0)[coord[a]], ok[coord[a]], ((t if o else 1.0 - t) != 0.0)[coord[a]]))
        pidx.append([p_[0] for p_ in per])
        inside.append([p_[1] for p_ in per])
        need.append([p_[2] for p_ in per])
    kinds = np.asarray(parent_kinds)
    for corner in range(8):
        o = (corner & 1, (corner >> 1) & 1, (corner >> 2) & 1)
        nd = need[0][o[0]] & need[1][o[1]] & need[2][o[2]]
        ins = inside[0][o[0]] & inside[1][o[1]] & inside[2][o[2]]
        if np.any(nd & ~ins):
            raise ValueError("a ghost cell's prior-mapping stencil leaves its parent box")
        pc = pidx[0][o[0]] + parent_shape[0] * (pidx[1][o[1]] + parent_shape[1] * pidx[2][o[2]])
        if np.any(nd & (kinds[pc] != FLUID)):
            raise ValueError("a ghost cell's prior-mapping stencil touches a non-fluid parent cell")


def check_shell_stencils(shell_shape, shell_origin, shell_dx, shell_cells,
                         src_kinds, src_shape, src_origin, src_dx, src_periodic):
    """The boundary shell of a scale, post-mapped from a far-field scale
    around it, must interpolate from cells of that scale that hold a state
    (not SOLID) inside its box on non-periodic axes."""
    nx, ny, _ = shell_shape
    gx, gy, gz = shell_cells % nx, (shell_cells // nx) % ny, shell_cells // (nx * ny)
    pts = np.stack([shell_origin[0] + gx * shell_dx, shell_origin[1] + gy * shell_dx,
                    shell_origin[2] + gz * shell_dx])
    base, t = _stencil(pts, src_origin, src_dx, src_shape)
    for corner in range(8):
        o = np.array([corner & 1, (corner >> 1) & 1, (corner >> 2) & 1])
        wt = np.ones(shell_cells.size)
        for a in range(3):
            wt *= t[a] if o[a] else 1.0 - t[a]
        idx = base + o[:, None]
        for a in range(3):
            if src_periodic & (1 << a):
                idx[a] %= src_shape[a]
        inside = np.all((idx >= 0) & (idx < np.array(src_shape)[:, None]), axis=0)
        need = wt != 0.0
        if np.any(need & ~inside):
            raise ValueError("a boundary cell's stencil leaves the far-field scale's box")
        sc = idx[0] + src_shape[0] * (idx[1] + src_shape[1] * idx[2])
        sc = np.where(inside, sc, 0)
        if np.any(need & (src_kinds[sc] == _capi.SOLID)):
            raise ValueError("a boundary cell's stencil touches a solid far-field cell")


def drop_overwritten_posts(post: dict, n: int, parents=None) -> dict:
    """Post-mapping lists {(fine i, coarse j): cells of j} with every cell
    removed that a later (finer) scale also post-maps into j.  Finer scales
    post-map in index order; when no scale after i reads j (prior-mapping
    reads the parent, and no later scale has j as its parent; far-field
    scales have taken their step before), a cell of j keeps only the later
    value, so leaving it out of i's list gives the same final state without
    the duplicate work.  ``parents`` (default: a chain, parent of k is
    k - 1) tells which later scales read j: if one does, i's list into j is
    kept whole, since that scale's prior-mappings see i's values."""
    if parents is None:
        parents = [-1] + list(range(n - 1))
    out = {}
    for j in range(n):
        keys = [i for i in range(n - 1, -1, -1) if i != j and (i, j) in post]
        if not keys:
            continue
        size = 1 + max(int(np.max(post[(i, j)])) if len(post[(i, j)]) else 0 for i in keys)
        later = np.zeros(size, bool)
        for i in keys:
            cells = np.asarray(post[(i, j)], np.int32)
            read_later = any(parents[k] == j for k in range(i + 1, n))
            out[(i, j)] = cells if read_later else cells[~later[cells]]
            later[cells] = True
    return out


POST_RUN = 256          # entries of a run: one workgroup of the tiled post-mapping
POST_TILE_BUFFER = 1280  # source cells of a run's box that fit in the kernel's LDS buffer
POST_TILE_MIN_FILL = 128  # mean entries a tile below which the direct gather is used: a
                          # workgroup stages its whole source box however few targets it maps


def post_tile_runs(cells: np.ndarray, shape, ratio: float, tile=None, order: str = "x"):
    """A post-mapping list into a dense box regrouped into tiles of
    neighbouring cells, and the run offsets of the tiles.

    A tile is tx x ty x tz cells (at most 256); a tile's cells are in box
    order.  order "x": the tiles follow each other x fastest, then y, then z
    (neighbouring runs share partly used source lines, which then meet in
    one L2: measured faster); "z": z fastest, then x, then y.  ``ratio`` is the spacing of the
    list's scale over that of the source scale (> 1).  Without ``tile``, tz
    is 1 and tx x ty is the first of 64 x 4, 64 x 2, 64 x 1, 32 x 2, ... whose
    source cells (at most floor((t - 1) * ratio) + 2 per axis, plus one for
    rounding, and 2 source planes) fit the kernel's buffer.  Returns (cells in tile order, int32 offsets
    with one entry more than there are tiles)."""
    c = np.asarray(cells, np.int32)   # cell indices of a level fit 32 bits
    nx, ny = shape[0], shape[1]
    if tile is None:
        # rows of 64 (one wavefront a row: whole-line stores, long source
        # rows) measured faster than squarer tiles that reach fewer source
        # cells per target; the deepest such tile that fits the buffer
        tz = 1
        for tx, ty in ((64, 4), (64, 2), (64, 1), (32, 2), (32, 1), (16, 1), (8, 1), (4, 1)):
            box = (math.floor((tx - 1) * ratio) + 3) * (math.floor((ty - 1) * ratio) + 3) * 2
            if box <= POST_TILE_BUFFER:
                break
    else:
        tx, ty, tz = tile
        assert tx * ty * tz <= POST_RUN
    x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
    kx, ky, kz = x // tx, y // ty, z // tz
    del x, y, z
    # one tile number per cell in the tiles' order, cells of a tile in box
    # order (a stable sort of a list that is in box order already)
    nkx, nky = int(kx.max(initial=0)) + 1, int(ky.max(initial=0)) + 1
    nkz = int(kz.max(initial=0)) + 1
    key = (ky * nkx + kx) * nkz + kz if order == "z" else (kz * nky + ky) * nkx + kx
    del kx, ky, kz
    if c.size < 2 or np.all(c[1:] > c[:-1]):
        order_idx = np.argsort(key, kind="stable")
    else:
        order_idx = np.lexsort((c, key))
    c = c[order_idx]
    key = key[order_idx]
    starts = np.flatnonzero(key[1:] != key[:-1]) + 1
    offsets = np.concatenate([[0], starts, [c.size]]).astype(np.int32)
    assert np.all(np.diff(offsets) <= POST_RUN)
    return c.astype(np.int32), offsets


POST_PLATE_KEEP = 0.75   # a plate tile is kept when at least this fraction of its cells is listed
SHELL_TILE_BUFFER = 512  # source cells of a ghost-shell patch's box that fit in the shell kernel's buffer


def _tile_source_cells(t, ratio: float) -> int:
    """Source cells the stencils of a tx x ty x tz tile can reach: per axis
    two planes for one target, else floor((t - 1) ratio) + 3 (one more for
    the rounding of the stencil base)."""
    n = 1
    for d in t:
        n *= 2 if d == 1 else math.floor((d - 1) * ratio) + 3
    return n


def _plate_tile(axis: int, ratio: float, depth: int = 2, buffer: int = POST_TILE_BUFFER):
    """The largest tile ``depth`` cells deep along ``axis`` (at most 256
    cells, its source box within ``buffer`` cells), longest along x
    first."""
    best = None
    for a in range(64, 0, -1):
        for b in range(min(POST_RUN // (depth * a), 64), 0, -1):
            t = [a, b]
            t.insert(axis, depth)
            if _tile_source_cells(t, ratio) <= buffer:
                key = (a * b, a)
                if best is None or key > best[0]:
                    best = (key, tuple(t))
                break
    return best[1]


def plate_tile_runs(cells: np.ndarray, shape, ratio: float):
    """A post-mapping list that lies in plates a few cells thick (the margin
    between nested boxes: the cells of scale 1 that scale 2 does not
    overwrite) regrouped into tiles lying in those plates.  For the plates
    normal to z, y and x in turn, tiles two, three or four cells deep along
    that axis (whichever keeps most; the largest tile of that depth whose
    source box fits the kernel's buffer, see _plate_tile) over a grid that
    starts at the smallest listed coordinate; a tile is kept when at least
    POST_PLATE_KEEP of it is listed.  What no plate tile keeps is cut, in
    blocks of 16 x 16 x 16 cells, into runs that end where the next cell
    would take the run's source box past the buffer.  Runs in the order of their first
    cell, each run's cells in box order.  Returns (cells in run order, int32
    offsets with one entry more than there are runs)."""
    c = np.asarray(cells, np.int64)
    nx, ny = shape[0], shape[1]
    xyz = (c % nx, (c // nx) % ny, c // (nx * ny))
    left = np.ones(c.size, bool)
    runs = []

    ascending = c.size < 2 or bool(np.all(c[1:] > c[:-1]))

    def tiles(idx, t):
        """the tiles of t over the entries idx that hold enough of them"""
        k = [(xyz[d][idx] - xyz[d][idx].min()) // t[d] for d in range(3)]
        key = (k[2] * (int(k[1].max()) + 1) + k[1]) * (int(k[0].max()) + 1) + k[0]
        # tiles in (z, y, x) order, each tile's cells in box order
        o = np.argsort(key, kind="stable") if ascending else np.lexsort((c[idx], key))
        idx = idx[o]
        key = key[o]
        st = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
        en = np.r_[st[1:], idx.size]
        keep = POST_PLATE_KEEP * t[0] * t[1] * t[2]
        return [idx[a:b] for a, b in zip(st, en) if b - a >= keep]

    for axis in (2, 1, 0):
        idx = np.flatnonzero(left)
        if idx.size == 0:
            break
        # plates two, three or four cells thick: the depth that keeps most
        best = max((tiles(idx, _plate_tile(axis, ratio, depth)) for depth in (2, 3, 4)),
                   key=lambda kept: sum(r.size for r in kept))
        for r in best:
            runs.append(r)
            left[r] = False
    rest = np.flatnonzero(left)
    if rest.size:
        # the rest (edges and strips that fill no tile) in blocks of 16^3,
        # each block's cells in box order, cut into runs as long as their
        # source box fits the buffer
        blk = [xyz[d][rest] // 16 for d in range(3)]
        rest = rest[np.lexsort((xyz[0][rest], xyz[1][rest], xyz[2][rest], blk[0], blk[1], blk[2]))]
        px, py, pz = (xyz[d][rest].tolist() for d in range(3))
        span = [2] + [math.floor(e * ratio) + 3 for e in range(1, max(shape) + 1)]   # by extent - 1
        start = 0
        x0 = x1 = px[0]
        y0 = y1 = py[0]
        z0 = z1 = pz[0]
        for k in range(1, rest.size):
            a0, a1 = min(x0, px[k]), max(x1, px[k])
            b0, b1 = min(y0, py[k]), max(y1, py[k])
            c0, c1 = min(z0, pz[k]), max(z1, pz[k])
            if k - start >= POST_RUN or span[a1 - a0] * span[b1 - b0] * span[c1 - c0] > POST_TILE_BUFFER:
                runs.append(np.sort(rest[start:k]))
                start = k
                x0 = x1 = px[k]
                y0 = y1 = py[k]
                z0 = z1 = pz[k]
            else:
                x0, x1, y0, y1, z0, z1 = a0, a1, b0, b1, c0, c1
        runs.append(np.sort(rest[start:]))
    runs.sort(key=lambda r: int(c[r[0]]))
    order = np.concatenate(runs) if runs else np.zeros(0, np.int64)
    offsets = np.cumsum([0] + [r.size for r in runs]).astype(np.int32)
    assert np.all(np.diff(offsets) <= POST_RUN)
    return c[order].astype(np.int32), offsets


def shell_tile_runs(cells: np.ndarray, shape, ratio: float, xface: bool = False):
    """Ghost cells of a one-cell shell regrouped into patches of its faces:
    tiles one cell deep of at most 256 cells whose source boxes fit the
    shell kernel's buffer of SHELL_TILE_BUFFER cells (64 x 4 at spacing
    ratios 3/4 and 2/3; see _plate_tile), over a grid that starts at the
    smallest listed coordinate.  A cell on the list's first or last z plane
    goes to a tile normal to z, else one on its first or last y plane to a
    tile normal to y, else one on its first or last x plane to a tile normal
    to x, else (not a shell cell) to a tile normal to z in its own plane;
    with ``xface`` (the entries of one of the shell's planes normal to x,
    which read a staged copy of the parent) every cell goes to a tile normal
    to x.  Every tile is a run, partly filled ones included.
    ``ratio`` is the shell's spacing over its parent's (< 1 for a finer
    scale).  Returns (cells in run order, int32 offsets with one entry more
    than there are runs)."""
    c = np.asarray(cells, np.int64)
    if c.size == 0:
        return c.astype(np.int32), np.zeros(1, np.int32)
    nx, ny = shape[0], shape[1]
    x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
    x, y, z = x - x.min(), y - y.min(), z - z.min()
    if xface:
        t = _plate_tile(0, ratio, 1, SHELL_TILE_BUFFER)
        key = [np.zeros_like(x), x, y // t[1], z // t[2]]
    else:
        tz = _plate_tile(2, ratio, 1, SHELL_TILE_BUFFER)
        ty = _plate_tile(1, ratio, 1, SHELL_TILE_BUFFER)
        tx = _plate_tile(0, ratio, 1, SHELL_TILE_BUFFER)
        on_z = (z == 0) | (z == z.max())
        on_y = ((y == 0) | (y == y.max())) & ~on_z
        # the x planes, when they are listed here too (no staged copies)
        on_x = ((x == 0) | (x == x.max())) & ~on_z & ~on_y
        face = np.where(on_x, 2, on_y.astype(np.int64))
        key = [face, np.select([on_x, on_y], [x, y], z),
               np.select([on_x, on_y], [y // tx[1], x // ty[0]], x // tz[0]),
               np.select([on_x, on_y], [z // tx[2], z // ty[2]], y // tz[1])]
    k = key[0]
    for part in key[1:]:
        k = k * (int(part.max()) + 1) + part
    order = np.lexsort((c, k))
    k = k[order]
    starts = np.flatnonzero(k[1:] != k[:-1]) + 1
    offsets = np.concatenate([[0], starts, [c.size]]).astype(np.int32)
    assert np.all(np.diff(offsets) <= POST_RUN)
    return c[order].astype(np.int32), offsets


def _nodes_coincide(src: Level, dst: Level) -> bool:
    """Every lattice point of dst is one of src (dst's spacing a whole
    multiple of src's, origins whole src cells apart): the library then maps
    each target from its one source point and uses no tile runs."""
    r = dst.c.dx / src.c.dx
    if r < 1.0 - 1e-9 or abs(r - round(r)) > 1e-9:
        return False
    return all(abs(o - round(o)) <= 1e-9 for o in
               ((dst.c.origin[d] - src.c.origin[d]) / src.c.dx for d in range(3)))


def _storage_list(lev: Level, box_cells: np.ndarray) -> np.ndarray:
    """A cell list over a level's box in the level's storage order (int32);
    every listed cell of a brick level must be stored."""
    if lev.dense_index is None:   # a dense box: storage order is box order
        return np.asarray(box_cells, np.int32)
    idx = lev.storage_of(np.asarray(box_cells, np.int64))
    if np.any(idx < 0):
        raise ValueError("a listed cell lies in a brick that is not stored")
    return idx.astype(np.int32)


class Hierarchy:
    """Scales 0..n-1 (0 = reference); parents[i] is the nearest coarser scale
    of a finer scale i (default i - 1).  A scale with a larger spacing than
    scale 0 is a far-field scale: its parent is the reference scale, its
    GHOST cells are the region it shares with it, and it post-maps onto the
    reference scale's GHOST shell.  A finer scale post-maps onto every
    larger scale: the scales before it and the far-field scales.  ``kinds`` are over each
    level's box (for a brick level: SOLID outside the stored bricks); the
    cell lists sent to the library are in each level's storage order.

    A post-mapping list from a finer dense scale into a coarser dense one is
    grouped into tiles (``tile_posts``) when they hold ``tile_min_fill``
    targets on average: plane tiles (post_tile_runs), or, where those are too
    sparse (``tile_plates`` "sparse"; "always": for every such list;
    "never"), tiles lying in the list's thin plates (plate_tile_runs).  The
    ghost shell of a dense scale in a dense, non-periodic parent is grouped
    into patches of its faces (``tile_shells``, shell_tile_runs) after its
    x-face entries."""

    def __init__(self, levels: list[Level], kinds: list[np.ndarray], parents=None, *,
                 stage_xfaces: bool = True, tile_posts: bool = True,
                 tile_min_fill: int = POST_TILE_MIN_FILL, tile_plates: str = "sparse",
                 tile_shells: bool = True):
        assert len(levels) == len(kinds) and 1 <= len(levels) <= _capi.MAX_SCALES
        self.levels = levels
        self.kinds = [np.asarray(k, np.uint8) for k in kinds]
        n = len(levels)
        self.far = [i > 0 and levels[i].c.dx > levels[0].c.dx for i in range(n)]
        if parents is None:
            parents, last_fine = [-1], 0
            for i in range(1, n):
                parents.append(0 if self.far[i] else last_fine)
                if not self.far[i]:
                    last_fine = i
        self.parents = list(parents)
        self.work = []
        self.lists = []
        self.stages = []
        self.post = {}
        far_post = {}
        self.c_scales = (_capi.CslbmScale * n)()
        dev = levels[0].device
        for i, lev in enumerate(levels):
            sc = self.c_scales[i]
            sc.parent = self.parents[i]
            work_f, work_g = [None, None], [None, None]
            if i > 0:
                work_f = [torch.zeros_like(lev.f), torch.zeros_like(lev.f)]
                if lev.g is not None:
                    work_g = [torch.zeros_like(lev.g), torch.zeros_like(lev.g)]
                ghosts = np.flatnonzero(self.kinds[i] == GHOST).astype(np.int32)
                par = levels[self.parents[i]]
                check_prior_stencils(self.kinds[self.parents[i]], (par.nx, par.ny, par.nz),
                                     tuple(par.c.origin), par.c.dx, par.c.periodic,
                                     (lev.nx, lev.ny, lev.nz), tuple(lev.c.origin), lev.c.dx, ghosts)
                if (stage_xfaces and not self.far[i] and lev.dense_index is None
                        and par.dense_index is None):
                    # ghosts on the shell's two planes normal to x first (each
                    # in (z, y) order): their prior-mapping reads a staged copy
                    # of the parent's columns around the plane
                    gx = ghosts % lev.nx
                    x_lo, x_hi = (int(gx.min()), int(gx.max())) if ghosts.size else (0, 0)
                    lo = gx == x_lo
                    hi = (gx == x_hi) & ~lo
                    ghosts = np.concatenate([ghosts[lo], ghosts[hi], ghosts[~(lo | hi)]])
                    par._sync_struct()
                    lev._sync_struct()
                    nb = int(_capi.load().cslbm_stage_bytes(C.byref(par.c), C.byref(lev.c), x_lo, x_hi))
                    if nb > 0:
                        st = torch.empty(nb, dtype=torch.uint8, device=dev)
                        self.stages.append(st)
                        sc.n_ghost_xlo, sc.n_ghost_xhi = int(lo.sum()), int(hi.sum())
                        sc.ghost_xlo, sc.ghost_xhi = x_lo, x_hi
                        sc.stage, sc.stage_bytes = st.data_ptr(), nb
                if (tile_shells and not self.far[i] and lev.dense_index is None
                        and par.dense_index is None and par.c.periodic == 0 and ghosts.size):
                    # the shell in patches of its faces, each mapped by one
                    # workgroup through LDS: each staged x plane's entries
                    # apart (they read that plane's copy), then the rest
                    ratio = lev.c.dx / par.c.dx
                    shape = (lev.nx, lev.ny)
                    parts, offs, at = [], [np.zeros(1, np.int32)], 0
                    bounds = np.cumsum([0, sc.n_ghost_xlo, sc.n_ghost_xhi, ghosts.size
                                        - sc.n_ghost_xlo - sc.n_ghost_xhi])
                    for k, (a, b) in enumerate(zip(bounds[:-1], bounds[1:])):
                        if b == a:
                            continue
                        t, r = shell_tile_runs(ghosts[a:b], shape, ratio, xface=k < 2)
                        parts.append(t)
                        offs.append(r[1:] + at)
                        at += t.size
                    ghosts = np.concatenate(parts).astype(np.int32)
                    runs = np.concatenate(offs).astype(np.int32)
                    r_t = torch.as_tensor(runs, device=dev)
                    self.lists.append(r_t)
                    sc.n_ghost_tiles = runs.size - 1
                    sc.ghost_tiles = r_t.data_ptr()
                g_t = torch.as_tensor(_storage_list(lev, ghosts), device=dev)
                self.lists.append(g_t)
                sc.n_ghost = ghosts.size
                sc.ghost_cells = g_t.data_ptr() if ghosts.size else None
                if self.far[i]:
                    # reversed rules: post-map onto the parent's boundary shell
                    pk = self.kinds[self.parents[i]]
                    shell = np.flatnonzero(pk == GHOST).astype(np.int32)
                    check_shell_stencils((par.nx, par.ny, par.nz), tuple(par.c.origin), par.c.dx,
                                         shell, self.kinds[i], (lev.nx, lev.ny, lev.nz),
                                         tuple(lev.c.origin), lev.c.dx, lev.c.periodic)
                    far_post[(i, self.parents[i])] = shell
                else:
                    # onto every larger scale: the scales before it and the
                    # far-field scales (section "Handling multiple scales")
                    for j in range(n):
                        if j == i or not (j < i or self.far[j]):
                            continue
                        cj = levels[j]
                        cells = post_cells(self.kinds[j], (cj.nx, cj.ny, cj.nz), tuple(cj.c.origin),
                                           cj.c.dx, self.kinds[i], (lev.nx, lev.ny, lev.nz),
                                           tuple(lev.c.origin), lev.c.dx)
                        self.post[(i, j)] = cells
            self.work.append((work_f, work_g))
            sc.work_f = (C.c_void_p * 2)(*[None if w is None else w.data_ptr() for w in work_f])
            sc.work_g = (C.c_void_p * 2)(*[None if w is None else w.data_ptr() for w in work_g])
        self.post_full = {**self.post, **far_post}
        self.post = {**drop_overwritten_posts(self.post, n, self.parents), **far_post}
        for (i, j), cells in self.post.items():
            if (tile_posts and cells.size and levels[i].dense_index is None
                    and levels[j].dense_index is None and levels[i].c.dx < levels[j].c.dx
                    and not _nodes_coincide(levels[i], levels[j])):
                # a finer dense scale into a coarser dense one: tiles of the
                # coarser box, each mapped by one workgroup through LDS
                ratio = levels[j].c.dx / levels[i].c.dx
                tiled, runs = post_tile_runs(cells, (levels[j].nx, levels[j].ny), ratio)
                if tile_plates == "always" or (tile_plates == "sparse" and
                                               tiled.size < tile_min_fill * (runs.size - 1)):
                    # too sparse for plane tiles: a list in thin plates
                    # fills tiles lying in those plates
                    tiled, runs = plate_tile_runs(cells, (levels[j].nx, levels[j].ny), ratio)
                if tiled.size >= tile_min_fill * (runs.size - 1):
                    cells = tiled
                    self.post[(i, j)] = cells
                    r_t = torch.as_tensor(runs, device=dev)
                    self.lists.append(r_t)
                    self.c_scales[i].n_post_tiles[j] = runs.size - 1
                    self.c_scales[i].post_tiles[j] = r_t.data_ptr()
            t = torch.as_tensor(_storage_list(levels[j], cells), device=dev)
            self.lists.append(t)
            self.c_scales[i].n_post[j] = cells.size
            self.c_scales[i].post_cells[j] = t.data_ptr() if cells.size else None
        self.c = _capi.CslbmHierarchy(n, 0, C.cast(self.c_scales, C.POINTER(_capi.CslbmScale)))

    def ghost_cells(self, i: int) -> np.ndarray:
        return np.flatnonzero(self.kinds[i] == GHOST).astype(np.int64)

    def step(self, n_ref: int = 1, stream=None):
        tensors = {}
        for i, lev in enumerate(self.levels):
            lev._sync_struct()
            self.c_scales[i].level = lev.c
            for t in (lev.f, lev.f_next, lev.g, lev.g_next, *self.work[i][0], *self.work[i][1]):
                if t is not None:
                    tensors[t.data_ptr()] = t
        _capi.call("cslbm_multiscale_step", C.byref(self.c), int(n_ref), _stream_handle(stream))
        for i, lev in enumerate(self.levels):
            sc = self.c_scales[i]
            lev.f = tensors[sc.level.f]
            lev.f_next = tensors[sc.level.f_next]
            if lev.g is not None:
                lev.g = tensors[sc.level.g]
                lev.g_next = tensors[sc.level.g_next]
            if i > 0:
                wf = [tensors[sc.work_f[0]], tensors[sc.work_f[1]]]
                wg = self.work[i][1]
                if lev.g is not None:
                    wg = [tensors[sc.work_g[0]], tensors[sc.work_g[1]]]
                self.work[i] = (wf, wg)
            lev._sync_struct()


    def _sync_scales(self):
        for i, lev in enumerate(self.levels):
            lev._sync_struct()
            self.c_scales[i].level = lev.c

    def adjoint_workspace_bytes(self) -> int:
        """Workspace bytes of adjoint_step (raises if the hierarchy is outside
        the adjoint's scope)."""
        self._sync_scales()
        lib = _capi.load()
        n = lib.cslbm_multiscale_adjoint_bytes(C.byref(self.c))
        if n < 0:
            raise _capi.CslbmError(_capi.ERR_UNSUPPORTED, "cslbm_multiscale_adjoint_bytes",
                                   lib.cslbm_last_error().decode())
        return int(n)

    def adjoint_step(self, f_in, g_in, lam, mu, workspace: torch.Tensor, stream=None):
        """Adjoint of one reference step (cslbm_multiscale_adjoint_step).
        f_in[i] / g_in[i]: scale i's state at t_n ([27][plane] / [7][plane]
        buffers); lam[i] / mu[i]: in dL/d(state at t_n + dt_0), out dL/d(state
        at t_n), overwritten in place."""
        self._sync_scales()
        n = len(self.levels)
        scalar = self.levels[0].g is not None
        vp = C.c_void_p * n
        ptrs = lambda ts: vp(*[t.data_ptr() for t in ts])  # noqa: E731
        _capi.call("cslbm_multiscale_adjoint_step", C.byref(self.c), ptrs(f_in),
                   ptrs(g_in) if scalar else None, ptrs(lam), ptrs(mu) if scalar else None,
                   workspace.data_ptr(), workspace.numel(), _stream_handle(stream))


# ---------------------------------------------------------------------------
# dynamic scale construction (section "Scale construction", dynamic scales)
# ---------------------------------------------------------------------------
def region_box(omega, speed, shape, thresholds, dilate: int, lo_limit, hi_limit):
    """Bounding box (inclusive level-0 cell bounds, x/y/z order) of the cells
    kept by the two thresholds of the dynamic construction, |curl u| >
    thresholds[0] and then |u| > thresholds[1], dilated by `dilate` cells
    and clipped to [lo_limit, hi_limit]; None when no cell passes."""
    nx, ny, nz = shape
    om = torch.as_tensor(omega)   # numpy or torch (then on its device)
    sp = torch.as_tensor(speed, device=om.device)
    w = ((om > thresholds[0]) & (sp > thresholds[1])).reshape(nz, ny, nx)
    # the bounding box from the three projections of the mask
    xs = np.flatnonzero(w.any(dim=1).any(dim=0).cpu().numpy())
    if xs.size == 0:
        return None
    ys = np.flatnonzero(w.any(dim=2).any(dim=0).cpu().numpy())
    zs = np.flatnonzero(w.any(dim=2).any(dim=1).cpu().numpy())
    lo = [int(xs[0]) - dilate, int(ys[0]) - dilate, int(zs[0]) - dilate]
    hi = [int(xs[-1]) + dilate, int(ys[-1]) + dilate, int(zs[-1]) + dilate]
    lo = [max(lo[a], lo_limit[a]) for a in range(3)]
    hi = [min(hi[a], hi_limit[a]) for a in range(3)]
    if any(h - l < 3 for l, h in zip(lo, hi)):
        return None
    return lo, hi


def fine_scale(lo, hi, alpha: float, params0: Params, solid_fn=None, *, scalar: bool,
               storage: int, row_align: int = 64):
    """A finer scale covering the level-0 box [lo, hi] (physical units of
    level 0) at spacing 1/alpha, anchored to the global lattice of that
    spacing.  Parameters: nu = alpha nu0, tau_s - 1/2 = alpha (tau_s0 - 1/2)
    (invariant local Reynolds and Peclet numbers).  Rows are padded to a
    multiple of `row_align` cells with SOLID cells beyond the ghost shell, so
    that every row starts on a cache-line boundary; no fluid cell ever pulls
    from them."""
    dx = 1.0 / alpha
    i0 = [math.ceil(lo[a] * alpha - 1e-9) for a in range(3)]
    i1 = [math.floor(hi[a] * alpha + 1e-9) for a in range(3)]
    inner_shape = tuple(i1[a] - i0[a] + 1 for a in range(3))
    nxp = -(-inner_shape[0] // row_align) * row_align
    shape = (nxp, inner_shape[1], inner_shape[2])
    origin = tuple(i0[a] * dx for a in range(3))
    # per-axis coordinates broadcast over the box (solid_fn is elementwise)
    k3 = np.zeros((shape[2], shape[1], shape[0]), np.uint8)
    if solid_fn is not None:
        px = origin[0] + np.arange(shape[0]) * dx
        py = origin[1] + np.arange(shape[1]) * dx
        pz = origin[2] + np.arange(shape[2]) * dx
        solid = np.broadcast_to(solid_fn(px[None, None, :], py[None, :, None], pz[:, None, None]),
                                k3.shape)
        k3[solid] = _capi.SOLID
    nx0 = inner_shape[0]
    k3[:, :, 0] = k3[:, :, nx0 - 1] = GHOST
    k3[:, 0, :] = k3[:, -1, :] = GHOST
    k3[0, :, :] = k3[-1, :, :] = GHOST
    k3[:, :, nx0:] = _capi.SOLID
    kinds = k3.reshape(-1)
    p = Params(**{**params0.__dict__})
    p.nu = params0.nu * alpha
    p.tau_s = 0.5 + alpha * (params0.tau_s - 0.5)
    lev = Level(*shape, p, storage=storage, scalar=scalar, periodic=0, flags=kinds,
                origin=origin, dx=dx)
    return lev, kinds


def brick_kinds(region: np.ndarray, solid: np.ndarray | None = None):
    """Stored bricks and cell kinds of a brick-stored scale.  ``region``
    (bool [nz][ny][nx], sizes multiples of 8) marks the cells the scale must
    cover; a brick is stored when it holds a region cell.  Stored cells with a
    neighbour (26-neighbourhood) outside the stored bricks or outside the box
    are GHOST (the scale's boundary, written by prior-mapping), the other
    stored cells FLUID, or SOLID where ``solid`` is set; cells outside the
    stored bricks are SOLID (never pulled: the ghost layer lies between).
    Returns (bricks [nz/8][ny/8][nx/8], kinds over the box)."""
    region = np.asarray(region, bool)
    nz, ny, nx = region.shape
    if nx % 8 or ny % 8 or nz % 8:
        raise ValueError(f"box {nx}x{ny}x{nz} is not a multiple of 8")
    bricks = region.reshape(nz // 8, 8, ny // 8, 8, nx // 8, 8).any(axis=(1, 3, 5))
    stored = bricks.repeat(8, 0).repeat(8, 1).repeat(8, 2)
    pad = np.pad(stored, 1, constant_values=False)
    inner = stored.copy()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                inner &= pad[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    kinds = np.full(stored.shape, _capi.SOLID, np.uint8)
    kinds[stored] = GHOST
    kinds[inner] = FLUID
    if solid is not None:
        kinds[inner & np.asarray(solid, bool).reshape(stored.shape)] = _capi.SOLID
    return bricks, kinds.reshape(-1)


def brick_scale_layout(lo, hi, alpha: float, region_fn, solid_fn=None):
    """Box, stored bricks and kinds of a brick-stored finer scale covering
    the level-0 box [lo, hi] at spacing 1/alpha (box sizes rounded up to
    multiples of 8): the bricks that hold cells where ``region_fn(px, py,
    pz)`` (physical coordinates, elementwise) is true, with the ghost layer
    of ``brick_kinds``.  Returns (shape, origin, dx, bricks, kinds)."""
    dx = 1.0 / alpha
    i0 = [math.ceil(lo[a] * alpha - 1e-9) for a in range(3)]
    i1 = [math.floor(hi[a] * alpha + 1e-9) for a in range(3)]
    shape = tuple(-(-(i1[a] - i0[a] + 1) // 8) * 8 for a in range(3))
    origin = tuple(i0[a] * dx for a in range(3))
    px = origin[0] + np.arange(shape[0]) * dx
    py = origin[1] + np.arange(shape[1]) * dx
    pz = origin[2] + np.arange(shape[2]) * dx
    full = (shape[2], shape[1], shape[0])
    region = np.broadcast_to(region_fn(px[None, None, :], py[None, :, None], pz[:, None, None]), full)
    solid = None
    if solid_fn is not None:
        solid = np.broadcast_to(solid_fn(px[None, None, :], py[None, :, None], pz[:, None, None]), full)
    bricks, kinds = brick_kinds(region, solid)
    return shape, origin, dx, bricks, kinds


def brick_scale(lo, hi, alpha: float, params0: Params, region_fn, solid_fn=None, *, scalar: bool,
                storage: int):
    """A finer scale like ``fine_scale`` stored in 8x8x8 bricks (see
    ``brick_scale_layout``).  Returns (level, kinds over the box)."""
    shape, origin, dx, bricks, kinds = brick_scale_layout(lo, hi, alpha, region_fn, solid_fn)
    p = Params(**{**params0.__dict__})
    p.nu = params0.nu * alpha
    p.tau_s = 0.5 + alpha * (params0.tau_s - 0.5)
    lev = Level(*shape, p, storage=storage, scalar=scalar, periodic=0, flags=kinds, origin=origin,
                dx=dx, bricks=bricks)
    return lev, kinds


def far_field_scale(ref: Level, ref_kinds: np.ndarray, dx: float, origin, shape, *,
                    periodic: int = 0, solid_fn=None):
    """A far-field scale (section "Scale construction": scales coarser than
    the reference over the far-field domain) of `shape` lattice points at
    origin + (x, y, z) * dx, dx > 1 in reference units (alpha_c = 1/dx).
    Cells whose trilinear stencil in the reference scale consists of its
    FLUID cells are GHOST (the shared region, mapped from the reference);
    faces on non-periodic axes are NEUMANN; `solid_fn` marks SOLID cells.
    Parameters: nu = alpha_c nu0, tau_s - 1/2 = alpha_c (tau_s0 - 1/2)."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    kinds = np.full(x.size, FLUID, np.uint8)
    if solid_fn is not None:
        kinds[solid_fn(origin[0] + x * dx, origin[1] + y * dx, origin[2] + z * dx)] = _capi.SOLID
    probe = np.where(kinds == FLUID, FLUID, _capi.SOLID).astype(np.uint8)
    shared = post_cells(probe, shape, tuple(origin), dx, np.asarray(ref_kinds, np.uint8),
                        (ref.nx, ref.ny, ref.nz), tuple(ref.c.origin), ref.c.dx)
    kinds[shared] = GHOST
    for a, (c, n) in enumerate(((x, nx), (y, ny), (z, nz))):
        if not periodic & (1 << a):
            kinds[((c == 0) | (c == n - 1)) & (kinds != _capi.SOLID)] = _capi.NEUMANN
    alpha = ref.c.dx / dx
    p = Params(**{**ref.params.__dict__})
    p.nu = ref.params.nu * alpha
    p.tau_s = 0.5 + alpha * (ref.params.tau_s - 0.5)
    lev = Level(nx, ny, nz, p, storage=ref.storage, scalar=ref.g is not None, periodic=periodic,
                flags=kinds, origin=tuple(origin), dx=dx)
    return lev, kinds


def fill_from_parent(parent: Level, lev: Level, stream=None):
    """Initialise every cell of a finer scale by mapping the parent's current
    state (full prior-mapping of a newly created region)."""
    cells = torch.arange(lev.n, dtype=torch.int32, device=lev.device)
    parent._sync_struct()
    lev._sync_struct()
    g_ok = parent.g is not None and lev.g is not None
    _capi.call("cslbm_exchange", C.byref(parent.c), parent.f.data_ptr(), None,
               parent.g.data_ptr() if g_ok else None, None, 0.0, C.byref(lev.c), lev.f.data_ptr(),
               lev.g.data_ptr() if g_ok else None, cells.data_ptr(), lev.n, _stream_handle(stream))


def kept_cells(old: Level, old_kinds: np.ndarray, new: Level, new_kinds: np.ndarray):
    """(old cells, new cells) of the FLUID cells two boxes of one scale share:
    both boxes lie on the global lattice of spacing dx (origins i0 dx), so a
    cell is the same lattice point in both when its global index matches."""
    dx = new.c.dx
    o_old = [int(round(old.c.origin[a] / dx)) for a in range(3)]
    o_new = [int(round(new.c.origin[a] / dx)) for a in range(3)]
    shp_old, shp_new = (old.nx, old.ny, old.nz), (new.nx, new.ny, new.nz)
    lo = [max(o_old[a], o_new[a]) for a in range(3)]
    hi = [min(o_old[a] + shp_old[a], o_new[a] + shp_new[a]) for a in range(3)]
    if any(h <= l for l, h in zip(lo, hi)):
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    # on the GPU when there is one (tens of millions of cells)
    dev = torch.device("cuda") if torch.cuda.is_available() else torch.device("cpu")
    gx, gy, gz = (torch.arange(lo[a], hi[a], device=dev) for a in range(3))

    def cells(o, shp):
        return ((gx - o[0])[None, None, :] +
                shp[0] * ((gy - o[1])[None, :, None] + shp[1] * (gz - o[2])[:, None, None])).reshape(-1)

    c_old, c_new = cells(o_old, shp_old), cells(o_new, shp_new)
    fl_old = torch.as_tensor(np.asarray(old_kinds) == FLUID, device=dev)
    fl_new = torch.as_tensor(np.asarray(new_kinds) == FLUID, device=dev)
    keep = fl_old[c_old] & fl_new[c_new]
    return (c_old[keep].to(torch.int32).cpu().numpy(), c_new[keep].to(torch.int32).cpu().numpy())


def copy_cells(src: Level, src_cells: np.ndarray, dst: Level, dst_cells: np.ndarray, stream=None):
    a = torch.as_tensor(np.asarray(src_cells, np.int32), device=dst.device)
    b = torch.as_tensor(np.asarray(dst_cells, np.int32), device=dst.device)
    src._sync_struct()
    dst._sync_struct()
    _capi.call("cslbm_copy_cells", C.byref(src.c), a.data_ptr(), C.byref(dst.c), b.data_ptr(),
               int(a.numel()), _stream_handle(stream))
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()


def _cube_dilate(m: torch.Tensor, r: int) -> torch.Tensor:
    """Dilation of a bool [nz][ny][nx] mask by the cube of half-width r
    (cells outside the array count as False): three 1-D max-pools, the same
    as r iterations with the 3x3x3 cube."""
    if r <= 0:
        return m
    dt = torch.float16 if m.is_cuda else torch.float32
    x = m.to(dt)[None, None]
    for k in ((2 * r + 1, 1, 1), (1, 2 * r + 1, 1), (1, 1, 2 * r + 1)):
        x = torch.nn.functional.max_pool3d(x, kernel_size=k, stride=1, padding=tuple(v // 2 for v in k))
    return x[0, 0] > 0


def _cube_erode(m: torch.Tensor, r: int) -> torch.Tensor:
    """Erosion of a bool mask by the cube of half-width r, cells outside the
    array counting as False (so the faces erode): the complement dilated,
    with the outside padded in."""
    if r <= 0:
        return m
    dt = torch.float16 if m.is_cuda else torch.float32
    x = torch.nn.functional.pad((~m).to(dt)[None, None], (r, r, r, r, r, r), value=1.0)
    for k in ((2 * r + 1, 1, 1), (1, 2 * r + 1, 1), (1, 1, 2 * r + 1)):
        x = torch.nn.functional.max_pool3d(x, kernel_size=k, stride=1)
    return ~(x[0, 0] > 0)


def object_labels(kinds0, shape) -> np.ndarray:
    """Connected components (face-connected) of the interior objects: SOLID
    cells of the reference scale off its box faces; 0 elsewhere."""
    nx, ny, nz = shape
    solid = np.asarray(kinds0).reshape(nz, ny, nx) == _capi.SOLID
    solid[:, :, [0, -1]] = False
    solid[:, [0, -1], :] = False
    solid[[0, -1], :, :] = False
    return ndimage.label(solid)[0]


def brick_regions(omega, speed, kinds0, shape, thresholds, alphas, *, margin: int = 3,
                  dilate: int = 2, nest: int = 2, labels=None):
    """Regions (bool [nz][ny][nx] over the reference scale) of brick-stored
    finer scales: the cells kept by each scale's thresholds, dilated; every
    interior object (SOLID cells off the box faces) that a region touches is
    added whole with a layer of fluid around it, thick enough to survive the
    shrinking of the deeper scales; then the region is cut to its parent's
    region shrunk by `nest` plus one brick of the scale (the reference: the
    box less `margin`), so that the scale's stored bricks and ghost layer lie
    on its parent's fluid.  Stops at the first empty region.  omega and speed
    may be torch tensors: the morphology then runs on their device.  `labels`
    (object_labels of kinds0) may be passed in when the geometry is reused."""
    nx, ny, nz = shape
    om = torch.as_tensor(omega).reshape(nz, ny, nx)
    sp = torch.as_tensor(speed, device=om.device).reshape(nz, ny, nx)
    dev = om.device
    if labels is None:
        labels = object_labels(kinds0, shape)
    lab = torch.as_tensor(labels, device=dev)
    # distances in the max norm (bricks and stencils are cubes)
    shrink = [nest + math.ceil(8 / a) for a in alphas]
    allowed = torch.zeros((nz, ny, nx), dtype=torch.bool, device=dev)
    allowed[margin:nz - margin, margin:ny - margin, margin:nx - margin] = True
    regions = []
    for k, thr in enumerate(thresholds):
        keep = (om > thr[0]) & (sp > thr[1])
        if not bool(keep.any()):
            break
        keep = _cube_dilate(keep, dilate)
        touched = torch.unique(lab[_cube_dilate(keep, 1) & (lab > 0)])
        if touched.numel():
            # the touched objects' cells (a lookup over the label values)
            hit = torch.zeros(int(lab.max()) + 1, dtype=torch.bool, device=dev)
            hit[touched.long()] = True
            keep |= _cube_dilate(hit[lab.long()], nest + 1 + sum(shrink[k + 1:]))
        region = keep & _cube_erode(allowed, shrink[k])
        if not bool(region.any()):
            break
        regions.append(region.cpu().numpy())
        allowed = region
    return regions


def region_box_fn(region: np.ndarray):
    """Bounding box (level-0 units, inclusive) of a region over the reference
    scale and its indicator at physical points (nearest reference cell)."""
    nz, ny, nx = region.shape
    zs, ys, xs = (np.flatnonzero(region.any(axis=ax)) for ax in ((1, 2), (0, 2), (0, 1)))
    lo = [int(xs[0]), int(ys[0]), int(zs[0])]
    hi = [int(xs[-1]), int(ys[-1]), int(zs[-1])]

    def region_fn(px, py, pz):
        ix = np.clip(np.rint(px).astype(np.int64), 0, nx - 1)
        iy = np.clip(np.rint(py).astype(np.int64), 0, ny - 1)
        iz = np.clip(np.rint(pz).astype(np.int64), 0, nz - 1)
        return region[iz, iy, ix]

    return lo, hi, region_fn


def dynamic_hierarchy(lev0: Level, kinds0: np.ndarray, thresholds, alphas, *, margin: int = 3,
                      dilate: int = 2, nest: int = 2, solid_fn=None, stream=None, previous=None,
                      bricks: bool = False, stage_xfaces: bool = True, tile_posts: bool = True):
    """Scales set by thresholds: scale k covers the bounding box of the cells
    with |curl u| > thresholds[k-1][0] and |u| > thresholds[k-1][1]
    (dilated), kept `margin` cells from the domain faces and `nest` cells
    inside its parent; spacing 1/alphas[k-1].  Returns (Hierarchy, boxes);
    scales whose region is empty are left out.

    With `previous` (a Hierarchy built by this function on the same
    reference scale) the regions are rebuilt, as the dynamic construction
    repeats every 40 iterations: every cell of a new scale first takes the
    full prior-mapping from its (new) parent, then the FLUID cells the old
    and the new box of that scale share keep their old state; cells that
    leave a region are dropped with the old levels.

    With `bricks` each finer scale stores only the 8x8x8 bricks holding its
    region (the cells kept by the thresholds, dilated, inside its parent's
    region shrunk by `nest` plus one brick of the scale, so that its stored
    bricks and their ghost layer lie on the parent's fluid), instead of the
    region's bounding box."""
    omega, speed = lev0.vorticity(stream)   # stay on the GPU: thresholds and morphology run there
    shape = (lev0.nx, lev0.ny, lev0.nz)
    lo_lim = [margin] * 3
    hi_lim = [shape[a] - 1 - margin for a in range(3)]
    levels, kinds, boxes = [lev0], [np.asarray(kinds0, np.uint8)], []
    labels = None
    if bricks:
        # the objects do not move: their labels are kept with the hierarchy
        old = getattr(previous, "object_labels", None)
        labels = old if old is not None and tuple(old.shape) == (shape[2], shape[1], shape[0]) \
            else torch.as_tensor(object_labels(kinds0, shape), device=omega.device)
    regions = brick_regions(omega, speed, kinds0, shape, thresholds, alphas, margin=margin,
                            dilate=dilate, nest=nest, labels=labels) if bricks else None
    for k_scale, (thr, alpha) in enumerate(zip(thresholds, alphas)):
        if bricks:
            if k_scale >= len(regions):
                break
            lo, hi, region_fn = region_box_fn(regions[k_scale])
            lev, k = brick_scale(lo, hi, alpha, lev0.params, region_fn, solid_fn,
                                 scalar=lev0.g is not None, storage=lev0.storage)
        else:
            box = region_box(omega, speed, shape, thr, dilate, lo_lim, hi_lim)
            if box is None:
                break
            lo, hi = box
            lev, k = fine_scale(lo, hi, alpha, lev0.params, solid_fn, scalar=lev0.g is not None,
                                storage=lev0.storage)
        fill_from_parent(levels[-1], lev, stream)
        i = len(levels)
        if previous is not None and i < len(previous.levels) and \
                abs(previous.levels[i].c.dx - lev.c.dx) < 1e-12:
            src, dst = kept_cells(previous.levels[i], previous.kinds[i], lev, k)
            # box indices to storage order (FLUID cells of a brick level are stored)
            copy_cells(previous.levels[i], _storage_list(previous.levels[i], src), lev,
                       _storage_list(lev, dst), stream)
        levels.append(lev)
        kinds.append(k)
        boxes.append((lo, hi))
        lo_lim = [lo[a] + nest for a in range(3)]
        hi_lim = [hi[a] - nest for a in range(3)]
    torch.cuda.synchronize()
    H = Hierarchy(levels, kinds, stage_xfaces=stage_xfaces, tile_posts=tile_posts)
    H.object_labels = labels
    return H, boxes


# ---------------------------------------------------------------------------
# static scale construction (section "Scale construction", static scales)
# ---------------------------------------------------------------------------
def object_distance(kinds: np.ndarray, shape, periodic: int = 0, faces: bool = True) -> np.ndarray:
    """Distance (reference cells) from every cell to the nearest SOLID cell or
    non-periodic box face, by an exact Euclidean distance transform.  With
    faces=False only objects count: SOLID cells on the box faces (walls)
    and the faces themselves are ignored."""
    nx, ny, nz = shape
    solid = np.asarray(kinds).reshape(nz, ny, nx) == _capi.SOLID
    if not faces:
        solid = solid.copy()
        solid[:, :, 0] = solid[:, :, -1] = False
        solid[:, 0, :] = solid[:, -1, :] = False
        solid[0, :, :] = solid[-1, :, :] = False
        if not solid.any():
            return np.full(nx * ny * nz, np.inf)
        periodic = 7
    free = ~solid
    pad = [(0 if periodic & (1 << a) else 1) for a in (2, 1, 0)]
    if any(pad):
        free = np.pad(free, [(p, p) for p in pad], constant_values=False)
    d = ndimage.distance_transform_edt(free)
    sl = tuple(slice(p, d.shape[i] - p) for i, p in enumerate(pad))
    return d[sl].reshape(-1)


def wake_shadow(kinds: np.ndarray, shape, inlet_center, inlet_radius: float, *,
                samples: int = 16, coarsen: int = 8) -> np.ndarray:
    """Soft shadow of the objects lit by the inlet disk on the x = 0 face (an
    area light): per cell, the fraction of `samples` points of the disk
    whose straight segment to the cell passes through a SOLID cell that is
    not on a box face.  1 in the umbra, between 0 and 1 in the penumbra.
    Computed on a grid coarsened by `coarsen` and sampled back."""
    nx, ny, nz = shape
    k = np.asarray(kinds).reshape(nz, ny, nx)
    obj = k == _capi.SOLID
    obj[:, :, 0] = obj[:, :, -1] = False
    obj[:, 0, :] = obj[:, -1, :] = False
    obj[0, :, :] = obj[-1, :, :] = False
    c = coarsen
    cz, cy, cx = -(-nz // c), -(-ny // c), -(-nx // c)
    occ = np.zeros((cz, cy, cx), bool)
    zz, yy, xx = np.nonzero(obj)
    occ[zz // c, yy // c, xx // c] = True
    # disk samples: a golden-angle spiral over the disk
    j = np.arange(samples) + 0.5
    rad = inlet_radius * np.sqrt(j / samples)
    ang = j * np.pi * (3.0 - np.sqrt(5.0))
    qy, qz = inlet_center[0] + rad * np.cos(ang), inlet_center[1] + rad * np.sin(ang)
    gz, gy, gx = np.meshgrid((np.arange(cz) + 0.5) * c, (np.arange(cy) + 0.5) * c,
                             (np.arange(cx) + 0.5) * c, indexing="ij")
    px, py, pz = gx.reshape(-1), gy.reshape(-1), gz.reshape(-1)
    hit = np.zeros(px.size)
    n_march = 2 * cx
    for s in range(samples):
        blocked = np.zeros(px.size, bool)
        for t in (np.arange(n_march) + 0.5) / n_march:
            x = t * px
            y = qy[s] + t * (py - qy[s])
            z = qz[s] + t * (pz - qz[s])
            ix = np.clip((x // c).astype(np.int64), 0, cx - 1)
            iy = np.clip((y // c).astype(np.int64), 0, cy - 1)
            iz = np.clip((z // c).astype(np.int64), 0, cz - 1)
            blocked |= occ[iz, iy, ix]
        hit += blocked
    frac = (hit / samples).reshape(cz, cy, cx)
    z, y, x = np.meshgrid(np.arange(nz) // c, np.arange(ny) // c, np.arange(nx) // c, indexing="ij")
    return frac[z, y, x].reshape(-1)


def static_levels(kinds: np.ndarray, shape, n_scales: int, d_max: float, *, periodic: int = 0,
                  faces: bool = True, inlet_center=None, inlet_radius: float = 0.0,
                  shadow_samples: int = 16, shadow_coarsen: int = 8) -> np.ndarray:
    """Scale index per cell (0 = the reference scale, n_scales - 1 = the
    finest): the distance to objects (and box faces unless faces=False),
    normalised by d_max and lowered in the objects' wake (soft shadow of
    the inlet), quantised into n_scales levels.  SOLID cells get level 0."""
    ind = np.clip(object_distance(kinds, shape, periodic, faces) / d_max, 0.0, 1.0)
    if inlet_center is not None and inlet_radius > 0.0:
        ind = np.minimum(ind, 1.0 - wake_shadow(kinds, shape, inlet_center, inlet_radius,
                                                samples=shadow_samples, coarsen=shadow_coarsen))
    lev = np.floor((1.0 - ind) * n_scales).astype(np.int64)
    lev = np.clip(lev, 0, n_scales - 1)
    lev[np.asarray(kinds) == _capi.SOLID] = 0
    return lev


def static_boxes(levels: np.ndarray, shape, n_scales: int, *, dilate: int = 2, margin: int = 3,
                 nest: int = 2):
    """Nested boxes (inclusive reference-cell bounds) of the cells at or
    above each level 1..n_scales-1; a level whose region is empty or
    degenerate ends the list."""
    nx, ny, nz = shape
    lv = levels.reshape(nz, ny, nx)
    lo_lim = [margin] * 3
    hi_lim = [shape[a] - 1 - margin for a in range(3)]
    boxes = []
    for k in range(1, n_scales):
        zs, ys, xs = np.nonzero(lv >= k)
        if xs.size == 0:
            break
        lo = [max(xs.min() - dilate, lo_lim[0]), max(ys.min() - dilate, lo_lim[1]),
              max(zs.min() - dilate, lo_lim[2])]
        hi = [min(xs.max() + dilate, hi_lim[0]), min(ys.max() + dilate, hi_lim[1]),
              min(zs.max() + dilate, hi_lim[2])]
        if any(h - l < 3 for l, h in zip(lo, hi)):
            break
        boxes.append((lo, hi))
        lo_lim = [lo[a] + nest for a in range(3)]
        hi_lim = [hi[a] - nest for a in range(3)]
    return boxes


def static_hierarchy(lev0: Level, kinds0: np.ndarray, n_scales: int, dx_min: float, d_max: float,
                     *, faces: bool = True, inlet_center=None, inlet_radius: float = 0.0,
                     solid_fn=None, stream=None, **kw):
    """Scales set by the domain geometry: levels from `static_levels`, boxes
    from `static_boxes`, spacings interpolated linearly from 1 (the
    reference) to dx_min (the finest), each scale filled from its parent.
    Returns (Hierarchy, boxes, spacings)."""
    shape = (lev0.nx, lev0.ny, lev0.nz)
    lv = static_levels(kinds0, shape, n_scales, d_max, periodic=lev0.c.periodic, faces=faces,
                       inlet_center=inlet_center, inlet_radius=inlet_radius)
    boxes = static_boxes(lv, shape, n_scales, **kw)
    spacings = [1.0 + (dx_min - 1.0) * k / (n_scales - 1) for k in range(1, n_scales)]
    levels, kinds = [lev0], [np.asarray(kinds0, np.uint8)]
    for (lo, hi), dx in zip(boxes, spacings):
        lev, k = fine_scale(lo, hi, 1.0 / dx, lev0.params, solid_fn, scalar=lev0.g is not None,
                            storage=lev0.storage)
        fill_from_parent(levels[-1], lev, stream)
        levels.append(lev)
        kinds.append(k)
    torch.cuda.synchronize()
    return Hierarchy(levels, kinds), boxes, spacings[:len(boxes)]
