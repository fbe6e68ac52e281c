// multiscale.hip -- cross-scale exchange, temporal interpolation and the
// reference-step driver (Algorithm 1) of libcslbm (gfx950).
//
// Exchange (eq. s1_to_s2_mapping): f~^dst = T(m^eq + K^ m~^neq,src) with
// K^ = (I - S^dst) K (I - S^src)^-1 and K = diag(S^src / (alpha S^dst)) on
// the stress moments m4..m8, 1 elsewhere.  In the central-moment frame of the
// interpolated state this touches only the second-order moments: the
// off-diagonal non-equilibrium k110, k101, k011 and the deviatoric part of
// the diagonal (m7 = k200 - k020, m8 = k200 - k002) are multiplied by
//   kappa = (1 - S_dst) / (1 - S_src) * S_src / (alpha S_dst),
// the trace (m9) and every other moment are carried over.  One thread per
// target cell; the 8-corner trilinear stencil (section "Spatial scale
// mapping") reads the source scale's states at two times and blends them
// with the time weight w (section "Temporal alignment and scale mapping").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

#include "../../include/cslbm.h"
#include "cm_collide.hpp"
#include "exchange.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "tile.hpp"

namespace cslbm {

// central-moment mapping of an interpolated post-collision state (in place,
// tensor order) and the stores of population and scalar outputs
template <typename Td>
__device__ __forceinline__ void map_and_store(const ExchArgs& a, int c, float (&v)[27],
                                              const float (&gi)[QS], bool scalar)
{
    float dr, jx, jy, jz;
    moments0(v, dr, jx, jy, jz);
    const float inv_rho = 1.0f / (1.0f + dr);
    const float ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    to_moments(v, ux, uy, uz);
    float d[27];
    deviation_equilibrium(d, dr, ux, uy, uz);
    const float kap = a.kappa;
    v[kslot(1, 1, 0)] = d[kslot(1, 1, 0)] + kap * (v[kslot(1, 1, 0)] - d[kslot(1, 1, 0)]);
    v[kslot(1, 0, 1)] = d[kslot(1, 0, 1)] + kap * (v[kslot(1, 0, 1)] - d[kslot(1, 0, 1)]);
    v[kslot(0, 1, 1)] = d[kslot(0, 1, 1)] + kap * (v[kslot(0, 1, 1)] - d[kslot(0, 1, 1)]);
    const float nxx = v[kslot(2, 0, 0)] - d[kslot(2, 0, 0)];
    const float nyy = v[kslot(0, 2, 0)] - d[kslot(0, 2, 0)];
    const float nzz = v[kslot(0, 0, 2)] - d[kslot(0, 0, 2)];
    const float tr = (nxx + nyy + nzz) * (1.0f / 3.0f);
    v[kslot(2, 0, 0)] = d[kslot(2, 0, 0)] + kap * (nxx - tr) + tr;
    v[kslot(0, 2, 0)] = d[kslot(0, 2, 0)] + kap * (nyy - tr) + tr;
    v[kslot(0, 0, 2)] = d[kslot(0, 0, 2)] + kap * (nzz - tr) + tr;
    from_moments(v, ux, uy, uz);

    Td* fo = static_cast<Td*>(a.fo);
#pragma unroll
    for (int i = 0; i < Q; ++i) Io<Td>::st(fo + i * a.dplane + c, v[tensor_slot(i)]);
    if (scalar) {
        const float s = (gi[0] + (gi[1] + gi[2])) + ((gi[3] + gi[4]) + (gi[5] + gi[6]));
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const float ge = kSw[i] * s * (1.0f + 4.0f * (kSx[i] * ux + kSy[i] * uy + kSz[i] * uz));
            a.go[i * a.dplane + c] = ge + a.kappa_s * (gi[i] - ge);
        }
    }
}

// Direct gather: each target reads its 8 source corners from global memory.
// kBlend reads both time levels and blends them with w; otherwise the host
// passes the one level that carries all the weight (w = 0 or w = 1).  Both
// switches are compile-time so that the 27 (or 54) loads of a corner carry no
// branch between them and are issued back to back.  Corners of zero weight
// are still read (at an index inside the box), without a branch.
// kNode: every target lies on a source lattice point (the host checked that
// the target spacing is an integer multiple of the source spacing and the
// origins differ by whole source cells), so the interpolation is the value
// at that point: one corner of weight 1 instead of eight.
// From a brick source, blocks run in XCD-contiguous order (xcd_block):
// neighbouring targets read the same source lines, which hold pieces of
// several bricks, and then meet in one L2 (a tenth of the lines fetched in
// natural order).  From a dense source the natural order is as fast or faster.
template <typename Ts, typename Td, bool kBlend, bool kScalar, bool kNode>
__global__ void __launch_bounds__(256) k_exchange(const ExchArgs a)
{
    int blk = a.sb.table ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    // the segment of this block (uniform: selected by the block index)
    const void* pA = a.fA;
    const void* pB = a.fB;
    const float* qA = a.gA;
    const float* qB = a.gB;
    int n[3] = {a.snx, a.sny, a.snz};
    int off[3] = {0, 0, 0};
    int64_t splane = a.splane;
    int first = a.main_first, count = a.n_cells - a.main_first;
    bool staged = false;
#pragma unroll
    for (int sgi = 0; sgi < 2; ++sgi) {
        if (staged || sgi >= a.n_staged) continue;
        if (blk < a.st[sgi].blocks) {
            const ExchArgs::Staged& g = a.st[sgi];
            pA = g.fA;
            pB = g.fB;
            qA = g.gA;
            qB = g.gB;
            n[0] = g.nx;
            n[1] = g.ny;
            n[2] = g.nz;
            off[0] = g.off[0];
            off[1] = g.off[1];
            off[2] = g.off[2];
            splane = g.plane;
            first = g.first;
            count = g.count;
            staged = true;
        } else {
            blk -= a.st[sgi].blocks;
        }
    }
    const int k = blk * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int c = a.cells[first + k];
    int base[3];
    float t[3];
    target_stencil(a, c, base, t);
#pragma unroll
    for (int d = 0; d < 3; ++d) base[d] -= off[d];
    if (kNode) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (t[d] >= 0.5f) ++base[d];   // nearest point (fractions are 0 up to rounding)
            t[d] = 0.0f;
        }
    }
    const int speriodic = staged ? 0 : a.speriodic;
    int ix[2], iy[2], iz[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        ix[o] = wrap_or_clamp(base[0] + o, n[0], speriodic & 1);
        iy[o] = wrap_or_clamp(base[1] + o, n[1], speriodic & 2);
        iz[o] = wrap_or_clamp(base[2] + o, n[2], speriodic & 4);
    }
    // A target on a source lattice plane (fraction 0 on that axis) gives the
    // upper corners weight 0: point them at the lower ones so that they hit
    // the cache lines just fetched instead of fetching a row nobody needs.
    // Branch-free, and the sum is unchanged (weight 0 times a finite value).
    if (t[0] == 0.0f) ix[1] = ix[0];
    if (t[1] == 0.0f) iy[1] = iy[0];
    if (t[2] == 0.0f) iz[1] = iz[0];
    // a staged copy holds the stencils of its face only
    const bool outside = staged && (base[0] < 0 || base[0] + 1 >= n[0] || base[1] < 0 ||
                                    base[1] + 1 >= n[1] || base[2] < 0 || base[2] + 1 >= n[2]);
    const Ts* fA = static_cast<const Ts*>(pA);
    const Ts* fB = static_cast<const Ts*>(pB);
    const float w = a.w;
    float v[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = 0.0f;
    float gi[QS] = {0, 0, 0, 0, 0, 0, 0};
    // Four corners per pass: their 136 (272 blended) loads are in flight
    // together.  All eight corners at once take more registers for no more
    // overlap; one corner at a time serialises eight round trips; both
    // measured slower.  The corners are summed in order 0..7 either way.
    constexpr int kCorners = kNode ? 1 : 8;
#pragma unroll 4
    for (int corner = 0; corner < kCorners; ++corner) {
        const int ox = corner & 1, oy = (corner >> 1) & 1, oz = (corner >> 2) & 1;
        const float wt = corner_weight(t, corner);
        const int cxi = ox ? ix[1] : ix[0], cyi = oy ? iy[1] : iy[0], czi = oz ? iz[1] : iz[0];
        const int64_t sc = staged ? cxi + (int64_t)n[0] * (cyi + (int64_t)n[1] * czi)
                                  : source_cell(a, cxi, cyi, czi);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float hA = Io<Ts>::ld(fA + i * splane + sc);
            if (kBlend) {
                const float hB = Io<Ts>::ld(fB + i * splane + sc);
                v[tensor_slot(i)] += wt * ((1.0f - w) * hA + w * hB);
            } else {
                v[tensor_slot(i)] += wt * hA;
            }
        }
        if (kScalar) {
#pragma unroll
            for (int i = 0; i < QS; ++i) {
                const float gA = qA[i * splane + sc];
                if (kBlend) {
                    const float gB = qB[i * splane + sc];
                    gi[i] += wt * ((1.0f - w) * gA + w * gB);
                } else {
                    gi[i] += wt * gA;
                }
            }
        }
    }
    if (outside) v[13] = __builtin_nanf("");
    map_and_store<Td>(a, c, v, gi, kScalar);
}

// Tiled exchange (tile.hpp): one workgroup maps one run of the list.
// Lanes past the run's end repeat its first entry: they compute the same
// bits as lane 0 and store them to the same cell.  kShell: runs that are
// patches of a ghost shell (small source boxes), blended or not; otherwise
// post-mapping runs (one time level).
template <typename Ts, typename Td, bool kScalar, bool kShell, bool kBlend>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_exchange_tiled(const ExchArgs a, const int32_t* runs)
{
    TileTarget T;
    float v[27], gi[QS];
    if constexpr (kShell) {
        __shared__ ShellLds lds;
        if (!tile_interp<Ts, kScalar, kBlend, kShellLoads, kShellPlanes, true>(a, runs, lds, T, v, gi))
            return;
    } else {
        __shared__ TileLds lds;
        if (!tile_interp<Ts, kScalar>(a, runs, lds, T, v, gi)) return;
    }
    map_and_store<Td>(a, T.c, v, gi, kScalar);
}

// Copy of sub-boxes of a dense level's two time levels (populations and
// scalar) into the compact staging layout: one thread per (face, plane,
// cell); cell k of face f's sub-box (x fastest) goes to element
// plane * S_f + k of that face's time-level blocks.
struct StageCopy {
    const void* fA;
    const void* fB;
    const float* gA;
    const float* gB;
    int64_t P;
    int pnx, pny;
    int planes;            // 27, or 34 with the scalar
    struct Face {
        int off[3], dim[3];
        int64_t S, cells, threads;   // threads = planes * cells
        void* oA;
        void* oB;
        float* ogA;
        float* ogB;
    } face[2];
};

template <typename T>
__global__ void __launch_bounds__(256) k_stage(const StageCopy a)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int f = 0;
    if (k >= a.face[0].threads) {
        k -= a.face[0].threads;
        f = 1;
        if (k >= a.face[1].threads) return;
    }
    const StageCopy::Face& F = a.face[f];
    const int pl = (int)(k / F.cells);
    const int64_t e = k - (int64_t)pl * F.cells;
    const int ix = (int)(e % F.dim[0]), iy = (int)((e / F.dim[0]) % F.dim[1]),
              iz = (int)(e / ((int64_t)F.dim[0] * F.dim[1]));
    const int64_t c = (F.off[0] + ix) + (int64_t)a.pnx * ((F.off[1] + iy) + (int64_t)a.pny * (F.off[2] + iz));
    if (pl < Q) {
        static_cast<T*>(F.oA)[pl * F.S + e] = static_cast<const T*>(a.fA)[pl * a.P + c];
        static_cast<T*>(F.oB)[pl * F.S + e] = static_cast<const T*>(a.fB)[pl * a.P + c];
    } else {
        const int s = pl - Q;
        F.ogA[s * F.S + e] = a.gA[s * a.P + c];
        F.ogB[s * F.S + e] = a.gB[s * a.P + c];
    }
}

// Lagrange quadratic in time, element by element over all planes
template <typename T>
__global__ void __launch_bounds__(256) k_time_interp(const T* s0, const T* s1, const T* s2,
                                                     T* out, const float* g0, const float* g1,
                                                     const float* g2, float* gout, int64_t N,
                                                     int64_t P, float l0, float l1, float l2)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    // nine planes at a time, all their loads before their stores (a store
    // between loads would order each later load after it; the output may be
    // one of the inputs, element for element)
#pragma unroll
    for (int i0 = 0; i0 < Q; i0 += 9) {
        float a[9], b[9], d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int64_t e = (i0 + i) * P + c;
            a[i] = Io<T>::ld(s0 + e);
            b[i] = Io<T>::ld(s1 + e);
            d[i] = Io<T>::ld(s2 + e);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) Io<T>::st(out + (i0 + i) * P + c, l0 * a[i] + l1 * b[i] + l2 * d[i]);
    }
    if (gout) {
        float a[QS], b[QS], d[QS];
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const int64_t e = i * P + c;
            a[i] = g0[e];
            b[i] = g1[e];
            d[i] = g2[e];
        }
#pragma unroll
        for (int i = 0; i < QS; ++i) gout[i * P + c] = l0 * a[i] + l1 * b[i] + l2 * d[i];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <typename Ts, typename Td>
static void launch_exchange_kernel(const ExchArgs& a, bool blend, bool scalar, bool node,
                                   dim3 grid, dim3 block, hipStream_t st)
{
    if (node && !blend) {
        if (scalar)
            hipLaunchKernelGGL((k_exchange<Ts, Td, false, true, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_exchange<Ts, Td, false, false, true>), grid, block, 0, st, a);
    } else if (blend && scalar)
        hipLaunchKernelGGL((k_exchange<Ts, Td, true, true, false>), grid, block, 0, st, a);
    else if (blend)
        hipLaunchKernelGGL((k_exchange<Ts, Td, true, false, false>), grid, block, 0, st, a);
    else if (scalar)
        hipLaunchKernelGGL((k_exchange<Ts, Td, false, true, false>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_exchange<Ts, Td, false, false, false>), grid, block, 0, st, a);
}

// Every target point of dst is a lattice point of src: the spacing ratio is
// a whole number and the origins differ by whole source cells.

static int launch_exchange_args(ExchArgs a, const cslbm_level* src, const cslbm_level* dst, double w,
                                hipStream_t stream)
{
    const bool scalar = a.gA != nullptr;
    // all the weight on one time level: read only that level
    const bool blend = w > 0.0 && w < 1.0;
    if (!blend && w >= 1.0) {
        a.fA = a.fB;
        a.gA = a.gB;
        for (int sgi = 0; sgi < a.n_staged; ++sgi) {
            a.st[sgi].fA = a.st[sgi].fB;
            a.st[sgi].gA = a.st[sgi].gB;
        }
    }
    const bool node = nodes_coincide(src, dst);
    int64_t blocks = (a.n_cells - a.main_first + 255) / 256;
    for (int sgi = 0; sgi < a.n_staged; ++sgi) blocks += a.st[sgi].blocks;
    if (blocks == 0) return CSLBM_OK;
    const dim3 grid((unsigned)blocks), block(256);
    const bool s32 = src->storage == CSLBM_F32, d32 = dst->storage == CSLBM_F32;
    if (s32 && d32)
        launch_exchange_kernel<float, float>(a, blend, scalar, node, grid, block, stream);
    else if (s32)
        launch_exchange_kernel<float, _Float16>(a, blend, scalar, node, grid, block, stream);
    else if (d32)
        launch_exchange_kernel<_Float16, float>(a, blend, scalar, node, grid, block, stream);
    else
        launch_exchange_kernel<_Float16, _Float16>(a, blend, scalar, node, grid, block, stream);
    return check_launch("k_exchange");
}

template <typename Ts, typename Td>
static void launch_tiled_kernel(const ExchArgs& a, const int32_t* runs, int32_t n_runs, bool shell,
                                bool blend, hipStream_t st)
{
    const dim3 grid((unsigned)n_runs), block(256);
    if (!shell) {
        if (a.gA)
            hipLaunchKernelGGL((k_exchange_tiled<Ts, Td, true, false, false>), grid, block, 0, st, a, runs);
        else
            hipLaunchKernelGGL((k_exchange_tiled<Ts, Td, false, false, false>), grid, block, 0, st, a, runs);
    } else if (blend) {
        if (a.gA)
            hipLaunchKernelGGL((k_exchange_tiled<Ts, Td, true, true, true>), grid, block, 0, st, a, runs);
        else
            hipLaunchKernelGGL((k_exchange_tiled<Ts, Td, false, true, true>), grid, block, 0, st, a, runs);
    } else {
        if (a.gA)
            hipLaunchKernelGGL((k_exchange_tiled<Ts, Td, true, true, false>), grid, block, 0, st, a, runs);
        else
            hipLaunchKernelGGL((k_exchange_tiled<Ts, Td, false, true, false>), grid, block, 0, st, a, runs);
    }
}

// one launch of the tiled kernel over runs of a's list (w in [0, 1]; a
// time weight strictly between blends the two levels, shell runs only)
static int launch_tiled(ExchArgs a, const cslbm_level* src, const cslbm_level* dst, double w,
                        const int32_t* runs, int32_t n_runs, bool shell, hipStream_t stream)
{
    const bool blend = w > 0.0 && w < 1.0;
    if (!blend && w >= 1.0) {
        a.fA = a.fB;
        a.gA = a.gB;
        for (int sgi = 0; sgi < a.n_staged; ++sgi) {
            a.st[sgi].fA = a.st[sgi].fB;
            a.st[sgi].gA = a.st[sgi].gB;
        }
    }
    const bool s32 = src->storage == CSLBM_F32, d32 = dst->storage == CSLBM_F32;
    if (s32 && d32)
        launch_tiled_kernel<float, float>(a, runs, n_runs, shell, blend, stream);
    else if (s32)
        launch_tiled_kernel<float, _Float16>(a, runs, n_runs, shell, blend, stream);
    else if (d32)
        launch_tiled_kernel<_Float16, float>(a, runs, n_runs, shell, blend, stream);
    else
        launch_tiled_kernel<_Float16, _Float16>(a, runs, n_runs, shell, blend, stream);
    return check_launch("k_exchange_tiled");
}

int launch_exchange(const cslbm_level* src, const void* fA, const void* fB, const float* gA,
                    const float* gB, double w, const cslbm_level* dst, void* f_out, float* g_out,
                    const int32_t* cells, int32_t n_cells, hipStream_t stream, const int32_t* runs,
                    int32_t n_runs)
{
    if (n_cells == 0) return CSLBM_OK;
    ExchArgs a = exchange_args(src, fA, fB, gA, gB, w, dst, f_out, g_out, cells, n_cells);
    const bool tiled = runs && n_runs > 0 && !(w > 0.0 && w < 1.0) && !a.sb.table && !a.db.table &&
                       a.speriodic == 0 && !nodes_coincide(src, dst);
    if (!tiled) return launch_exchange_args(a, src, dst, w, stream);
    return launch_tiled(a, src, dst, w, runs, n_runs, false, stream);
}

// ---------------------------------------------------------------------------
// x-face staging of a ghost shell's prior-mapping.  A target on a box face
// x = const reads 2 cells of each of 4 parent rows per plane: from the
// parent's x-fastest planes that is one cache line per 8 useful bytes, and
// neighbouring targets (along y) read different rows.  Copying the parent's
// few columns around the face into a compact sub-box once per reference
// step (both time levels) lets those targets read contiguous memory.
// ---------------------------------------------------------------------------
struct StageFace {
    int off[3], dim[3];
    int64_t S;          // elements per plane (sub-box cells rounded up to 64)
    int64_t bytes;
    int64_t popB, gA, gB;   // byte offsets of the sections in the face's block
};

struct StagePlan {
    StageFace face[2];
    int64_t bytes;
};

static int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Sub-boxes of parent P holding the stencils of L's shell planes x = x_lo
// and x = x_hi (one cell of margin on every side for the rounding of the
// stencil base); false when staging does not apply.
static bool stage_plan(const cslbm_level* P, const cslbm_level* L, int x_lo, int x_hi, StagePlan* sp)
{
    sp->bytes = 0;
    if (P->brick_table || L->brick_table) return false;
    if (x_lo < 0 || x_hi < x_lo || x_hi >= L->nx) return false;
    const int64_t esz = P->storage == CSLBM_F32 ? 4 : 2;
    const bool scalar = L->g != nullptr;
    const int pn[3] = {P->nx, P->ny, P->nz};
    const int ln[3] = {L->nx, L->ny, L->nz};
    for (int f = 0; f < 2; ++f) {
        StageFace& F = sp->face[f];
        int64_t cells = 1;
        for (int d = 0; d < 3; ++d) {
            double qa, qb;
            if (d == 0) {
                const int xf = f == 0 ? x_lo : x_hi;
                qa = qb = (L->origin[0] + xf * L->dx - P->origin[0]) / P->dx;
            } else {
                qa = (L->origin[d] - P->origin[d]) / P->dx;
                qb = (L->origin[d] + (ln[d] - 1) * L->dx - P->origin[d]) / P->dx;
            }
            int lo = (int)std::floor(qa) - 1, hi = (int)std::floor(qb) + 2;
            if (lo < 0 || hi > pn[d] - 1) {
                if (P->periodic & (1 << d)) return false;   // the stencils wrap
                lo = std::max(lo, 0);
                hi = std::min(hi, pn[d] - 1);
            }
            if (hi < lo) return false;
            F.off[d] = lo;
            F.dim[d] = hi - lo + 1;
            cells *= F.dim[d];
        }
        F.S = (cells + 63) / 64 * 64;
        const int64_t pop = align256(Q * F.S * esz), gs = scalar ? align256(QS * F.S * 4) : 0;
        F.popB = pop;
        F.gA = 2 * pop;
        F.gB = 2 * pop + gs;
        F.bytes = 2 * pop + 2 * gs;
        sp->bytes += F.bytes;
    }
    return true;
}

// copy both faces' sub-boxes of the parent's states A and B into the stage
// (one launch; one thread per face, plane and cell)
static int stage_faces(const cslbm_level* P, const StagePlan& sp, const void* A, const void* B,
                       const float* gA, const float* gB, char* stage, hipStream_t stream)
{
    StageCopy c;
    c.fA = A;
    c.fB = B;
    c.gA = gA;
    c.gB = gB;
    c.P = P->plane;
    c.pnx = P->nx;
    c.pny = P->ny;
    c.planes = gA ? Q + QS : Q;
    char* base = stage;
    int64_t threads = 0;
    for (int f = 0; f < 2; ++f) {
        const StageFace& F = sp.face[f];
        StageCopy::Face& G = c.face[f];
        for (int d = 0; d < 3; ++d) {
            G.off[d] = F.off[d];
            G.dim[d] = F.dim[d];
        }
        G.S = F.S;
        G.cells = (int64_t)F.dim[0] * F.dim[1] * F.dim[2];
        G.threads = c.planes * G.cells;
        G.oA = base;
        G.oB = base + F.popB;
        G.ogA = gA ? reinterpret_cast<float*>(base + F.gA) : nullptr;
        G.ogB = gA ? reinterpret_cast<float*>(base + F.gB) : nullptr;
        threads += G.threads;
        base += F.bytes;
    }
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    if (P->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_stage<float>, grid, block, 0, stream, c);
    else
        hipLaunchKernelGGL(k_stage<_Float16>, grid, block, 0, stream, c);
    return check_launch("k_stage");
}

static void set_stage_segments(const StagePlan& sp, char* stage, int32_t n_xlo, int32_t n_xhi, ExchArgs& a);

// Prior-mapping of a shell whose list starts with the n_xlo + n_xhi ghosts
// of its two planes normal to x: those read the staged copies (one segment
// per plane), the rest the parent itself, all in one launch.
static int launch_prior_staged(const cslbm_level* P, const StagePlan& sp, char* stage, const void* A,
                               const void* B, const float* gA, const float* gB, double w,
                               const cslbm_level* dst, void* f_out, float* g_out, const int32_t* cells,
                               int32_t n_xlo, int32_t n_xhi, int32_t n_cells, hipStream_t stream)
{
    if (n_cells == 0) return CSLBM_OK;
    ExchArgs a = exchange_args(P, A, B, gA, gB, w, dst, f_out, g_out, cells, n_cells);
    set_stage_segments(sp, stage, n_xlo, n_xhi, a);
    return launch_exchange_args(a, P, dst, w, stream);
}

// The staged segments of a shell's list (the n_xlo + n_xhi x-face entries
// first) over the faces of plan sp in stage; the scalar sections only when
// a carries the scalar.
static void set_stage_segments(const StagePlan& sp, char* stage, int32_t n_xlo, int32_t n_xhi, ExchArgs& a)
{
    const bool scalar = a.gA != nullptr;
    char* face = stage;
    int first = 0;
    a.n_staged = 2;
    for (int f = 0; f < 2; ++f) {
        const StageFace& F = sp.face[f];
        ExchArgs::Staged& g = a.st[f];
        g.fA = face;
        g.fB = face + F.popB;
        g.gA = scalar ? reinterpret_cast<const float*>(face + F.gA) : nullptr;
        g.gB = scalar ? reinterpret_cast<const float*>(face + F.gB) : nullptr;
        g.nx = F.dim[0];
        g.ny = F.dim[1];
        g.nz = F.dim[2];
        for (int d = 0; d < 3; ++d) g.off[d] = F.off[d];
        g.plane = F.S;
        g.first = first;
        g.count = f == 0 ? n_xlo : n_xhi;
        g.blocks = (g.count + 255) / 256;
        first += g.count;
        face += F.bytes;
    }
    a.main_first = first;
}

bool prior_segments(const cslbm_scale& sc, bool staged, const cslbm_level* P, ExchArgs& a)
{
    StagePlan sp;
    if (!staged || !stage_plan(P, &sc.level, sc.ghost_xlo, sc.ghost_xhi, &sp)) return false;
    set_stage_segments(sp, static_cast<char*>(sc.stage), sc.n_ghost_xlo, sc.n_ghost_xhi, a);
    return true;
}

int prior_stage(const cslbm_scale& sc, const cslbm_level* P, const void* A, const void* B,
                const float* gA, const float* gB, bool* staged, hipStream_t stream)
{
    StagePlan sp;
    *staged = sc.stage && sc.n_ghost_xlo + sc.n_ghost_xhi > 0 &&
              stage_plan(P, &sc.level, sc.ghost_xlo, sc.ghost_xhi, &sp);
    return *staged ? stage_faces(P, sp, A, B, gA, gB, static_cast<char*>(sc.stage), stream) : CSLBM_OK;
}

// The ghost shell's entries after its x faces go in patch runs through LDS
// (cslbm_scale.ghost_tiles): dense boxes, no periodic parent axis, targets
// off the parent's lattice points.
static bool shell_tiled(const cslbm_scale& sc, const cslbm_level* P)
{
    const cslbm_level* L = &sc.level;
    return sc.ghost_tiles && sc.n_ghost_tiles > 0 && !P->brick_table && !L->brick_table &&
           P->periodic == 0 && !nodes_coincide(P, L);
}

int prior_map(const cslbm_scale& sc, bool staged, const cslbm_level* P, const void* A, const void* B,
              const float* gA, const float* gB, double w, void* out, float* gout, hipStream_t stream)
{
    const cslbm_level* L = &sc.level;
    StagePlan sp;
    const bool stage = staged && stage_plan(P, L, sc.ghost_xlo, sc.ghost_xhi, &sp);
    if (shell_tiled(sc, P)) {
        // every run in one launch; runs of x-face entries read the staged
        // copies when there are any
        if (sc.n_ghost == 0) return CSLBM_OK;
        ExchArgs a = exchange_args(P, A, B, gA, gB, w, L, out, gout, sc.ghost_cells, sc.n_ghost);
        if (stage) set_stage_segments(sp, static_cast<char*>(sc.stage), sc.n_ghost_xlo, sc.n_ghost_xhi, a);
        return launch_tiled(a, P, L, w, sc.ghost_tiles, sc.n_ghost_tiles, true, stream);
    }
    if (!stage) return launch_exchange(P, A, B, gA, gB, w, L, out, gout, sc.ghost_cells, sc.n_ghost, stream);
    return launch_prior_staged(P, sp, static_cast<char*>(sc.stage), A, B, gA, gB, w, L, out, gout,
                               sc.ghost_cells, sc.n_ghost_xlo, sc.n_ghost_xhi, sc.n_ghost, stream);
}

static int launch_time_interp(const cslbm_level* L, const void* s0, const void* s1, const void* s2,
                              const float* g0, const float* g1, const float* g2, const double t[3],
                              double te, void* out, float* g_out, hipStream_t stream)
{
    const double l0 = (te - t[1]) * (te - t[2]) / ((t[0] - t[1]) * (t[0] - t[2]));
    const double l1 = (te - t[0]) * (te - t[2]) / ((t[1] - t[0]) * (t[1] - t[2]));
    const double l2 = (te - t[0]) * (te - t[1]) / ((t[2] - t[0]) * (t[2] - t[1]));
    const int64_t N = cells_of(L);
    const bool scalar = g0 && g1 && g2 && g_out;
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_time_interp<float>, grid, block, 0, stream, (const float*)s0,
                           (const float*)s1, (const float*)s2, (float*)out, scalar ? g0 : nullptr,
                           g1, g2, scalar ? g_out : nullptr, N, L->plane, (float)l0, (float)l1,
                           (float)l2);
    else
        hipLaunchKernelGGL(k_time_interp<_Float16>, grid, block, 0, stream, (const _Float16*)s0,
                           (const _Float16*)s1, (const _Float16*)s2, (_Float16*)out,
                           scalar ? g0 : nullptr, g1, g2, scalar ? g_out : nullptr, N, L->plane,
                           (float)l0, (float)l1, (float)l2);
    return check_launch("k_time_interp");
}

static int validate_exchange_pair(const cslbm_level* src, const cslbm_level* dst)
{
    int rc = validate_shape(src);
    if (rc) return rc;
    rc = validate_shape(dst);
    if (rc) return rc;
    if (!(src->dx > 0.0) || !(dst->dx > 0.0))
        return fail(CSLBM_ERR_ARG, "scale spacings must be positive (src %g, dst %g)", src->dx, dst->dx);
    if (!(src->p.nu > 0.0) || !(dst->p.nu > 0.0))
        return fail(CSLBM_ERR_ARG, "scale viscosities must be positive");
    const double Ss = shear_rate(src);
    if (std::fabs(1.0 - Ss) < 1e-9)
        return fail(CSLBM_ERR_ARG, "source relaxation time is 1: (I - S)^-1 of the mapping is singular");
    return CSLBM_OK;
}

// a scale with a larger spacing than the reference scale (far field)
static bool far_field(const cslbm_scale* S, int i) { return i > 0 && S[i].level.dx > S[0].level.dx; }

// Checks of a hierarchy shared by the multi-scale step and its adjoint.
int validate_hierarchy(const cslbm_hierarchy* H)
{
    if (!H || !H->scales) return fail(CSLBM_ERR_ARG, "hierarchy is NULL");
    const int ns = H->n_scales;
    if (ns < 1 || ns > CSLBM_MAX_SCALES)
        return fail(CSLBM_ERR_ARG, "n_scales = %d outside [1, %d]", ns, CSLBM_MAX_SCALES);
    const cslbm_scale* S = H->scales;
    const bool scalar = S[0].level.g != nullptr;
    for (int i = 0; i < ns; ++i) {
        const cslbm_level* L = &S[i].level;
        int rc = validate_shape(L);
        if (rc) return fail(rc, "scale %d: %s", i, cslbm_last_error());
        rc = validate_params(L);
        if (rc) return fail(rc, "scale %d: %s", i, cslbm_last_error());
        if (!L->f_next || L->f == L->f_next) return fail(CSLBM_ERR_ARG, "scale %d: bad f_next", i);
        if (L->p.grad_mode != 0)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: the gradient mode is single-level only", i);
        if ((L->g != nullptr) != scalar)
            return fail(CSLBM_ERR_ARG, "scale %d: every scale or none must carry the scalar", i);
        if (!(L->dx > 0.0)) return fail(CSLBM_ERR_ARG, "scale %d: dx must be positive", i);
        if (std::fabs(1.0 - shear_rate(L)) < 1e-9)
            return fail(CSLBM_ERR_ARG, "scale %d: relaxation time 1 makes the mapping singular", i);
        if (scalar && std::fabs(L->p.tau_s - 1.0) < 1e-9)
            return fail(CSLBM_ERR_ARG, "scale %d: scalar relaxation time 1 is singular", i);
        if (i == 0) {
            if (S[0].parent != -1) return fail(CSLBM_ERR_ARG, "scale 0 must have parent -1");
            continue;
        }
        if (S[i].parent < 0 || S[i].parent >= i)
            return fail(CSLBM_ERR_ARG, "scale %d: parent %d must be a scale with index < %d", i,
                        S[i].parent, i);
        const cslbm_level* PL = &S[S[i].parent].level;
        if (far_field(S, i)) {
            if (S[i].parent != 0)
                return fail(CSLBM_ERR_ARG, "far-field scale %d: its parent must be the reference scale", i);
            if (!(PL->dx < L->dx))
                return fail(CSLBM_ERR_ARG, "far-field scale %d is not coarser than its parent", i);
            for (int j = 0; j < ns; ++j)
                if (j != S[i].parent && S[i].n_post[j] != 0)
                    return fail(CSLBM_ERR_ARG,
                                "far-field scale %d may post-map only onto its parent's shell", i);
        } else {
            if (far_field(S, S[i].parent))
                return fail(CSLBM_ERR_ARG, "scale %d: a finer scale's parent cannot be a far-field scale", i);
            if (!(L->dx <= PL->dx))
                return fail(CSLBM_ERR_ARG, "scale %d is not finer than its parent", i);
            for (int j = i; j < ns; ++j)
                if (!far_field(S, j) && S[i].n_post[j] != 0)
                    return fail(CSLBM_ERR_ARG,
                                "scale %d may post-map only onto larger scales (index < %d or far field), not %d",
                                i, i, j);
        }
        if (!L->flags) return fail(CSLBM_ERR_ARG, "scale %d: needs flags (ghost cells)", i);
        if (!S[i].work_f[0] || !S[i].work_f[1])
            return fail(CSLBM_ERR_ARG, "scale %d: two work buffers are required", i);
        if (scalar && (!S[i].work_g[0] || !S[i].work_g[1]))
            return fail(CSLBM_ERR_ARG, "scale %d: two scalar work buffers are required", i);
        if (S[i].n_ghost < 0 || (S[i].n_ghost > 0 && !S[i].ghost_cells))
            return fail(CSLBM_ERR_ARG, "scale %d: bad ghost list", i);
        for (int j = 0; j < ns; ++j) {
            if (S[i].n_post[j] < 0 || (S[i].n_post[j] > 0 && !S[i].post_cells[j]))
                return fail(CSLBM_ERR_ARG, "scale %d: bad post-mapping list for scale %d", i, j);
            if (S[i].n_post_tiles[j] < 0 || S[i].n_post_tiles[j] > S[i].n_post[j] ||
                (S[i].n_post_tiles[j] > 0 && !S[i].post_tiles[j]))
                return fail(CSLBM_ERR_ARG, "scale %d: bad run offsets of the post-mapping list for scale %d",
                            i, j);
        }
        if (S[i].n_ghost_tiles < 0 || S[i].n_ghost_tiles > S[i].n_ghost ||
            (S[i].n_ghost_tiles > 0 && !S[i].ghost_tiles))
            return fail(CSLBM_ERR_ARG, "scale %d: bad run offsets of the ghost list", i);
        if (S[i].n_ghost_xlo < 0 || S[i].n_ghost_xhi < 0 ||
            (int64_t)S[i].n_ghost_xlo + S[i].n_ghost_xhi > S[i].n_ghost)
            return fail(CSLBM_ERR_ARG, "scale %d: x-face ghost counts %d + %d exceed the %d ghosts", i,
                        S[i].n_ghost_xlo, S[i].n_ghost_xhi, S[i].n_ghost);
        if (S[i].stage && !far_field(S, i)) {
            StagePlan sp;
            if (stage_plan(PL, L, S[i].ghost_xlo, S[i].ghost_xhi, &sp) && S[i].stage_bytes < sp.bytes)
                return fail(CSLBM_ERR_ARG, "scale %d: stage of %lld bytes, %lld needed", i,
                            (long long)S[i].stage_bytes, (long long)sp.bytes);
        }
    }

    return CSLBM_OK;
}

}  // namespace cslbm

using namespace cslbm;

extern "C" {

int cslbm_exchange(const cslbm_level* src, const void* fA, const void* fB, const float* gA,
                   const float* gB, double w, const cslbm_level* dst, void* f_out, float* g_out,
                   const int32_t* cells, int32_t n_cells, hipStream_t stream)
{
    int rc = validate_exchange_pair(src, dst);
    if (rc) return rc;
    if (!fA || !f_out) return fail(CSLBM_ERR_ARG, "source or destination populations are NULL");
    if (n_cells < 0 || (n_cells > 0 && !cells)) return fail(CSLBM_ERR_ARG, "bad cell list");
    if (!(w >= 0.0 && w <= 1.0)) return fail(CSLBM_ERR_ARG, "time weight %g outside [0, 1]", w);
    if (g_out && gA && std::fabs(src->p.tau_s - 1.0) < 1e-9)
        return fail(CSLBM_ERR_ARG, "source scalar relaxation time is 1 (singular mapping)");
    return launch_exchange(src, fA, fB, gA, gB, w, dst, f_out, g_out, cells, n_cells, stream);
}

int64_t cslbm_stage_bytes(const cslbm_level* parent, const cslbm_level* level, int32_t x_lo,
                          int32_t x_hi)
{
    int rc = validate_shape(parent);
    if (rc) return rc;
    rc = validate_shape(level);
    if (rc) return rc;
    if (!(parent->dx > 0.0) || !(level->dx > 0.0))
        return fail(CSLBM_ERR_ARG, "scale spacings must be positive");
    StagePlan sp;
    return stage_plan(parent, level, x_lo, x_hi, &sp) ? sp.bytes : 0;
}

int cslbm_time_interp(const cslbm_level* L, const void* s0, const void* s1, const void* s2,
                      const float* g0, const float* g1, const float* g2, const double t[3],
                      double t_eval, void* out, float* g_out, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!s0 || !s1 || !s2 || !out || !t) return fail(CSLBM_ERR_ARG, "NULL state or times");
    if (t[0] == t[1] || t[0] == t[2] || t[1] == t[2])
        return fail(CSLBM_ERR_ARG, "interpolation times must be distinct");
    return launch_time_interp(L, s0, s1, s2, g0, g1, g2, t, t_eval, out, g_out, stream);
}


int cslbm_multiscale_step(cslbm_hierarchy* H, int32_t n_ref_steps, hipStream_t stream)
{
    int vrc = validate_hierarchy(H);
    if (vrc) return vrc;
    if (n_ref_steps < 0) return fail(CSLBM_ERR_ARG, "n_ref_steps is negative");
    const int ns = H->n_scales;
    cslbm_scale* S = H->scales;
    // states of each scale at t_n (A) and t_n + dt_0 (B) within one reference step
    const void* A[CSLBM_MAX_SCALES];
    void* B[CSLBM_MAX_SCALES];
    const float* gA[CSLBM_MAX_SCALES];
    float* gB[CSLBM_MAX_SCALES];
    for (int n = 0; n < n_ref_steps; ++n) {
        // reference scale: one step (Algorithm 1, first statement of the loop)
        {
            cslbm_level* L = &S[0].level;
            int rc = launch_step_into(L, L->f, L->f_next, L->g, L->g_next, stream);
            if (rc) return rc;
            std::swap(L->f, L->f_next);
            std::swap(L->g, L->g_next);
            A[0] = L->f_next;
            B[0] = L->f;
            gA[0] = L->g_next;
            gB[0] = L->g;
        }
        // far-field scales (spacing larger than the reference scale) advance
        // with the reference scale, before the finer scales (Algorithm 1),
        // with the reversed rules of section "Handling multiple scales": the
        // whole region shared with the parent (GHOST cells of this scale) is
        // mapped from the parent at t_n, the scale takes one step of
        // dt_c = dt_0 / alpha_c and is interpolated linearly back to
        // t_n + dt_0 (fused into the step's store), the shared region is
        // mapped again at t_n + dt_0, and the parent's boundary shell is
        // post-mapped from this scale.
        for (int i = 1; i < ns; ++i) {
            if (!far_field(S, i)) continue;
            cslbm_scale& sc = S[i];
            cslbm_level* L = &sc.level;
            const cslbm_level* P = &S[sc.parent].level;
            const int p = sc.parent;
            const double ac = S[0].level.dx / L->dx;
            void* X0 = L->f;
            float* gX0 = L->g;
            void* R = sc.work_f[1];
            float* gR = sc.work_g[1];
            int rc = launch_exchange(P, A[p], B[p], gA[p], gB[p], 0.0, L, X0, gX0, sc.ghost_cells,
                                     sc.n_ghost, stream);
            if (rc) return rc;
            rc = launch_step_interp(L, X0, R, gX0, gR, X0, gX0, 1.0 - ac, 0.0, ac, stream);
            if (rc) return rc;
            rc = launch_exchange(P, A[p], B[p], gA[p], gB[p], 1.0, L, R, gR, sc.ghost_cells,
                                 sc.n_ghost, stream);
            if (rc) return rc;
            A[i] = X0;
            B[i] = R;
            gA[i] = gX0;
            gB[i] = gR;
            rc = launch_exchange(L, R, R, gR, gR, 0.0, P, B[p], gB[p], sc.post_cells[p], sc.n_post[p],
                                 stream);
            if (rc) return rc;
        }
        // finer scales, coarse to fine
        for (int i = 1; i < ns; ++i) {
            if (far_field(S, i)) continue;
            cslbm_scale& sc = S[i];
            cslbm_level* L = &sc.level;
            const cslbm_level* P = &S[sc.parent].level;
            const int p = sc.parent;
            const double alpha = S[0].level.dx / L->dx;
            const int l = (int)std::floor(alpha + 1e-12) + 1;
            void* X0 = L->f;
            void* bufs[2] = {L->f_next, sc.work_f[0]};
            float* gX0 = L->g;
            float* gbufs[2] = {L->g_next, sc.work_g[0]};
            void* cur = X0;
            float* gcur = gX0;
            // the quadratic through 0, (l-1)/alpha, l/alpha evaluated at 1,
            // fused into the last sub-step's output
            const double t[3] = {0.0, (l - 1) / alpha, l / alpha};
            const double L0 = (1.0 - t[1]) * (1.0 - t[2]) / ((t[0] - t[1]) * (t[0] - t[2]));
            const double L1 = (1.0 - t[0]) * (1.0 - t[2]) / ((t[1] - t[0]) * (t[1] - t[2]));
            const double L2 = (1.0 - t[0]) * (1.0 - t[1]) / ((t[2] - t[0]) * (t[2] - t[1]));
            // At integer alpha the middle node is t = 1 itself: the quadratic
            // has weights (0, 1, 0) there and the last sub-step does not enter
            // the result (in floating point too: 0 * a + 1 * b + 0 * c == b).
            // It is then not computed: the state after sub-step l - 1 is the
            // interpolated state, and its ghosts are mapped at weight 1 below
            // just as the skipped sub-step's prior-mapping would have done.
            const bool node = L2 == 0.0 && L0 == 0.0 && L1 == 1.0;
            const int last = node ? l - 1 : l;
            void* R = sc.work_f[1];
            float* gR = sc.work_g[1];
            // x-face ghosts read a staged copy of the parent's columns around
            // each face (both time levels, copied once per reference step)
            bool staged = false;
            {
                int rc = prior_stage(sc, P, A[p], B[p], gA[p], gB[p], &staged, stream);
                if (rc) return rc;
            }
            for (int k = 1; k <= last; ++k) {
                // prior-mapping of the boundary shell: the parent blended at
                // the sub-step's start time, or at t_n + dt_0 before the last
                int rc = prior_map(sc, staged, P, A[p], B[p], gA[p], gB[p], prior_weight(k, l, alpha),
                                   cur, gcur, stream);
                if (rc) return rc;
                if (k < l) {
                    const int slot = (k - 1) & 1;
                    void* next = bufs[slot];
                    float* gnext = gbufs[slot];
                    if (node && k == last) {   // the result goes straight to R
                        next = R;
                        gnext = gR;
                    }
                    rc = launch_step_into(L, cur, next, gcur, gnext, stream);
                    if (rc) return rc;
                    cur = next;
                    gcur = gnext;
                } else {
                    rc = launch_step_interp(L, cur, R, gcur, gR, X0, gX0, L0, L1, L2, stream);
                    if (rc) return rc;
                }
            }
            int rc = prior_map(sc, staged, P, A[p], B[p], gA[p], gB[p], 1.0, R, gR, stream);
            if (rc) return rc;
            A[i] = X0;
            B[i] = R;
            gA[i] = gX0;
            gB[i] = gR;
            // post-mapping onto every larger scale, far-field scales included
            // (section "Handling multiple scales"), in index order
            for (int j = 0; j < ns; ++j) {
                if (j == i || sc.n_post[j] == 0) continue;
                rc = launch_exchange(L, R, R, gR, gR, 0.0, &S[j].level, B[j], gB[j],
                                     sc.post_cells[j], sc.n_post[j], stream, sc.post_tiles[j],
                                     sc.n_post_tiles[j]);
                if (rc) return rc;
            }
        }
        // the interpolated states become the scales' states at the new reference time
        for (int i = 1; i < ns; ++i) {
            std::swap(S[i].level.f, S[i].work_f[1]);
            std::swap(S[i].level.g, S[i].work_g[1]);
        }
    }
    return CSLBM_OK;
}

}  // extern "C"
