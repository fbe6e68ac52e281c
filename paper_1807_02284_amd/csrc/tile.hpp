// tile.hpp -- trilinear gather of one run of exchange targets through LDS
// (section "Spatial scale mapping"), shared by the tiled post-mapping and
// its adjoint.
//
// Dense source and destination, no periodic source axis, targets off the
// source lattice points.  One workgroup takes one run of the target list
// (the host groups neighbouring cells of the destination into runs of at
// most 256: a tile of a few rows).  The source cells the run's stencils
// reach form a small box (a 32 x 8 x 1 tile at spacing ratio 4/3 reaches at
// most 44 x 12 x 2 of them); the workgroup copies that box into LDS a few
// population planes at a time with row-wise coalesced loads, and each
// target then takes its 8 corners from LDS.  Gathered from global memory
// instead, every source line is requested by the 2 x-corners of each of the
// (about 1.5 x 1.5) target rows that reach it and each time it is touched
// partially.  Corner order and arithmetic are those of the direct gather,
// so the interpolated states are bitwise the same.  A run whose box exceeds
// the buffer is gathered directly.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include <climits>

#include "exchange.hpp"
#include "internal.hpp"
#include "lattice.hpp"

namespace cslbm {

constexpr int kTileCap = 1280;                // floats per plane buffer
constexpr int kTileLoads = kTileCap / 256;    // buffer elements per thread
constexpr int kTilePlanes = 4;                // planes staged per barrier round trip
// Patches of a ghost shell (one cell thick, targets finer than the source):
// their boxes hold at most 512 cells (a 64 x 4 patch at spacing ratio 3/4
// reaches 50 x 5 x 2), so two buffer elements a thread and eight planes per
// round trip in a quarter of the LDS.
constexpr int kShellLoads = 2;
constexpr int kShellPlanes = 8;

__device__ __forceinline__ uint32_t raw_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t raw_bits(_Float16 v) { return __builtin_bit_cast(uint16_t, v); }

template <typename T>
__device__ __forceinline__ float from_bits(uint32_t b);
template <>
__device__ __forceinline__ float from_bits<float>(uint32_t b)
{
    return __uint_as_float(b);
}
template <>
__device__ __forceinline__ float from_bits<_Float16>(uint32_t b)
{
    return static_cast<float>(__builtin_bit_cast(_Float16, (uint16_t)b));
}

template <int kLoads, int kPlanes>
struct TileBuf {
    static constexpr int kCap = 256 * kLoads;   // floats per plane buffer
    float buf[kPlanes * kCap];
    int box[6];
};
using TileLds = TileBuf<kTileLoads, kTilePlanes>;
using ShellLds = TileBuf<kShellLoads, kShellPlanes>;

// One target of a run: its cell, list index, stencil base and fractions,
// and its corner indices along each axis (the upper one equal to the lower
// where the fraction is 0).  Lanes past the run's end take its first entry.
struct TileTarget {
    int c, k;
    bool active;
    int base[3], lo[3], hi[3];
    float t[3];
};

// Interpolated state of this thread's target (v in tensor order, gi the
// scalar) from the time level a.fA / a.gA, or with kBlend from both levels
// blended with a.w as the direct gather does it per corner (here per
// source cell on its way into LDS: the same value).  Returns false, for
// every thread of the workgroup, when the run is empty.  Every thread fills its
// kLoads buffer slots without a branch (past the box it reloads the
// box's last cell): predicated fills made the compiler version the unrolled
// plane loop.  Each plane's corner sum is pinned where it is computed (an
// empty asm reads it): a caller whose stores are conditional otherwise had
// the sums sunk past the barriers, with all 8 x 34 corner values live.
// kStaged: a run whose first entry lies in a staged segment of a (the
// x-face copies of a ghost shell's prior-mapping) reads that copy, with the
// corner indices shifted as in the direct gather, and a target whose
// stencil leaves the copy becomes NaN as there; runs must not mix segments.
template <typename Ts, bool kScalar, bool kBlend = false, int kLoads = kTileLoads,
          int kPlanes = kTilePlanes, bool kStaged = false>
__device__ __forceinline__ bool tile_interp(const ExchArgs& a, const int32_t* runs,
                                            TileBuf<kLoads, kPlanes>& L, TileTarget& T,
                                            float (&v)[27], float (&gi)[QS])
{
    constexpr int kCap = TileBuf<kLoads, kPlanes>::kCap;
    // runs in tile order: every XCD walks one contiguous range of them, so
    // the source planes that neighbouring runs share meet in one L2.  A
    // shell's runs in dispatch order instead: its x-face runs come first,
    // and their scattered stores (one cache line per cell and plane) go
    // to every XCD rather than to the first.
    const int r = kStaged ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
    const int start = max(runs[r], 0), end = min(runs[r + 1], a.n_cells);
    const int count = min(end - start, 256);
    if (count <= 0) return false;   // uniform over the workgroup
    const int tid = threadIdx.x;
    T.active = tid < count;
    T.k = start + (T.active ? tid : 0);
    T.c = a.cells[T.k];
    target_stencil(a, T.c, T.base, T.t);
    // the run's source: a staged copy or the source level (uniform)
    const void* pA = a.fA;
    const void* pB = a.fB;
    const float* pgA = a.gA;
    const float* pgB = a.gB;
    int n[3] = {a.snx, a.sny, a.snz};
    int64_t P = a.splane;
    bool outside = false;
    if constexpr (kStaged) {
        int off[3] = {0, 0, 0};
        bool staged = false;
#pragma unroll
        for (int sgi = 0; sgi < 2; ++sgi) {
            const ExchArgs::Staged& g = a.st[sgi];
            if (!staged && sgi < a.n_staged && start >= g.first && start < g.first + g.count) {
                pA = g.fA;
                pB = g.fB;
                pgA = g.gA;
                pgB = g.gB;
                n[0] = g.nx;
                n[1] = g.ny;
                n[2] = g.nz;
                off[0] = g.off[0];
                off[1] = g.off[1];
                off[2] = g.off[2];
                P = g.plane;
                staged = true;
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            T.base[d] -= off[d];
            outside |= staged && (T.base[d] < 0 || T.base[d] + 1 >= n[d]);
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T.lo[d] = wrap_or_clamp(T.base[d], n[d], false);
        T.hi[d] = T.t[d] == 0.0f ? T.lo[d] : wrap_or_clamp(T.base[d] + 1, n[d], false);
    }
    // the run's source box: block-wide min of lo and max of hi
    if (tid < 6) L.box[tid] = tid < 3 ? INT_MAX : INT_MIN;
    __syncthreads();
    int m[6] = {T.lo[0], T.lo[1], T.lo[2], T.hi[0], T.hi[1], T.hi[2]};
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const int o = __shfl_xor(m[d], s);
            m[d] = d < 3 ? min(m[d], o) : max(m[d], o);
        }
    if ((tid & 63) == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            atomicMin(&L.box[d], m[d]);
            atomicMax(&L.box[d + 3], m[d + 3]);
        }
    }
    __syncthreads();
    const int x0 = L.box[0], y0 = L.box[1], z0 = L.box[2];
    const int bx = L.box[3] - x0 + 1, by = L.box[4] - y0 + 1, bz = L.box[5] - z0 + 1;
    const int V = bx * by * bz;
    const Ts* fA = static_cast<const Ts*>(pA);
    const Ts* fB = static_cast<const Ts*>(pB);
    const float* qA = pgA;
    const float* qB = pgB;
    const float w = a.w;
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = 0.0f;
#pragma unroll
    for (int i = 0; i < QS; ++i) gi[i] = 0.0f;
    if (V > kCap) {   // uniform: direct gather
#pragma unroll 1   // one corner at a time: this rare path must not raise the register count
        for (int corner = 0; corner < 8; ++corner) {
            const float wt = corner_weight(T.t, corner);
            const int cx = corner & 1 ? T.hi[0] : T.lo[0], cy = corner & 2 ? T.hi[1] : T.lo[1];
            const int cz = corner & 4 ? T.hi[2] : T.lo[2];
            const int64_t sc = cx + (int64_t)n[0] * (cy + (int64_t)n[1] * cz);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const float hA = Io<Ts>::ld(fA + i * P + sc);
                if constexpr (kBlend) {
                    const float hB = Io<Ts>::ld(fB + i * P + sc);
                    v[tensor_slot(i)] += wt * ((1.0f - w) * hA + w * hB);
                } else {
                    v[tensor_slot(i)] += wt * hA;
                }
            }
            if (kScalar)
#pragma unroll
                for (int i = 0; i < QS; ++i) {
                    if constexpr (kBlend)
                        gi[i] += wt * ((1.0f - w) * qA[i * P + sc] + w * qB[i * P + sc]);
                    else
                        gi[i] += wt * qA[i * P + sc];
                }
        }
        if (outside) v[13] = __builtin_nanf("");
        return true;
    }
    // source offsets of this thread's box elements (the same in every plane)
    const int64_t origin = x0 + (int64_t)n[0] * (y0 + (int64_t)n[1] * z0);
    int eoff[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int e = min(tid + 256 * k, V - 1);
        const int ex = e % bx, ey = (e / bx) % by, ez = e / (bx * by);
        eoff[k] = ex + n[0] * (ey + n[1] * ez);
    }
    int cl[8];
    float wt[8];
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
        const int cx = corner & 1 ? T.hi[0] : T.lo[0], cy = corner & 2 ? T.hi[1] : T.lo[1];
        const int cz = corner & 4 ? T.hi[2] : T.lo[2];
        cl[corner] = (cx - x0) + bx * ((cy - y0) + by * (cz - z0));
        wt[corner] = corner_weight(T.t, corner);
    }
    // kPlanes planes per phase: one barrier round trip moves that many
    // planes, and the next phase's loads are in flight while this phase is
    // summed from LDS
    constexpr int NP = kScalar ? Q + QS : Q;
    constexpr int NG = (NP + kPlanes - 1) / kPlanes;
    // binary16 elements stay raw bits until the LDS write: converted where
    // they were loaded, each load was waited for before the next was issued
    constexpr bool kHalf = std::is_same<Ts, _Float16>::value;
    using Pre = typename std::conditional<kHalf, uint32_t, float>::type;
    constexpr int kLevels = kBlend ? 2 : 1;
    Pre pre[kLevels][kPlanes][kLoads];
    auto fetch = [&](int grp) {
#pragma unroll
        for (int lv = 0; lv < kLevels; ++lv) {
            const Ts* f = lv ? fB : fA;
            const float* q = lv ? qB : qA;
#pragma unroll
            for (int p = 0; p < kPlanes; ++p) {
                const int i = grp * kPlanes + p;
                if (i < NP)
#pragma unroll
                    for (int k = 0; k < kLoads; ++k) {
                        if constexpr (kHalf)
                            pre[lv][p][k] = i < Q ? raw_bits(*(f + i * P + origin + eoff[k]))
                                                  : raw_bits(q[(i - Q) * P + origin + eoff[k]]);
                        else
                            pre[lv][p][k] = i < Q ? Io<Ts>::ld(f + i * P + origin + eoff[k])
                                                  : q[(i - Q) * P + origin + eoff[k]];
                    }
            }
        }
    };
    // an element as it was loaded, as a float
    auto value = [&](int lv, int p, int k, bool pop) -> float {
        if constexpr (kHalf)
            return pop ? from_bits<_Float16>(pre[lv][p][k]) : from_bits<float>(pre[lv][p][k]);
        else
            return pre[lv][p][k];
    };
    fetch(0);
#pragma unroll
    for (int grp = 0; grp < NG; ++grp) {
        if (grp) __syncthreads();   // every thread has summed the previous phase
#pragma unroll
        for (int p = 0; p < kPlanes; ++p)
            if (grp * kPlanes + p < NP)
#pragma unroll
                for (int k = 0; k < kLoads; ++k) {
                    const bool pop = grp * kPlanes + p < Q;
                    if constexpr (kBlend) {
                        const float hA = value(0, p, k, pop), hB = value(1, p, k, pop);
                        L.buf[p * kCap + tid + 256 * k] = (1.0f - w) * hA + w * hB;
                    } else {
                        L.buf[p * kCap + tid + 256 * k] = value(0, p, k, pop);
                    }
                }
        __syncthreads();
        if (grp + 1 < NG) fetch(grp + 1);
#pragma unroll
        for (int p = 0; p < kPlanes; ++p) {
            const int i = grp * kPlanes + p;
            if (i >= NP) continue;
            float s = 0.0f;
#pragma unroll
            for (int corner = 0; corner < 8; ++corner) s += wt[corner] * L.buf[p * kCap + cl[corner]];
            asm volatile("" : : "v"(s));
            if (i < Q)
                v[tensor_slot(i)] = s;
            else
                gi[i - Q] = s;
        }
    }
    if (outside) v[13] = __builtin_nanf("");
    return true;
}

}  // namespace cslbm
