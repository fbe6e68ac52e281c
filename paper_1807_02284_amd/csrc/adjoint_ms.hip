// adjoint_ms.hip -- reverse mode of one reference step of Algorithm 1 over a
// chain of finer scales (gfx950): the adjoints of the exchange (prior- and
// post-mapping, section "Handling multiple scales"), of the quadratic time
// interpolation fused into the last sub-step (section "Temporal alignment and
// scale mapping") and of every collide-stream step, in the reverse order of
// the forward schedule.
//
// The forward step is recomputed from the scales' states at t_n into a
// caller-provided workspace (the input of every sub-step and the
// interpolated result), then walked backwards.  Post-mapped values are never
// read again within a reference step when every scale's parent is the next
// coarser scale, so the recompute leaves them out and the adjoint of a
// post-mapping only routes the target cells' adjoint to the fine state and
// clears it there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/cslbm.h"
#include "cm_adjoint.hpp"
#include "cm_collide.hpp"
#include "exchange.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "tile.hpp"

namespace cslbm {

// Vector-Jacobian product of the exchange's cell map: the interpolated
// post-collision state v (tensor order) and scalar gi go to
//   out = K(u)^-1 (k with its second-order non-equilibrium rescaled by kappa,
//                  the trace kept),  k = K(u) v, u = j / (1 + dr),
//   g_out = g^eq(s, u) + kappa_s (gi - g^eq(s, u)),  s = sum gi.
// Given lam = dL/d(out) and mu = dL/d(g_out), returns vb = dL/dv and
// gb = dL/dgi.
template <bool kScalar>
__device__ __forceinline__ void exchange_map_adjoint(const float (&v)[27], const float (&gi)[7],
                                                     float kap, float kap_s,
                                                     const float (&lam)[27], const float (&mu)[7],
                                                     float (&vb)[27], float (&gb)[7])
{
    float dr, jx, jy, jz;
    moments0(v, dr, jx, jy, jz);
    const float ir = 1.0f / (1.0f + dr);
    const float ux = jx * ir, uy = jy * ir, uz = jz * ir;

    // forward: mapped moments w
    float w[27];
    {
        float d[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) w[q] = v[q];
        to_moments(w, ux, uy, uz);
        deviation_equilibrium(d, dr, ux, uy, uz);
        w[kslot(1, 1, 0)] = d[kslot(1, 1, 0)] + kap * (w[kslot(1, 1, 0)] - d[kslot(1, 1, 0)]);
        w[kslot(1, 0, 1)] = d[kslot(1, 0, 1)] + kap * (w[kslot(1, 0, 1)] - d[kslot(1, 0, 1)]);
        w[kslot(0, 1, 1)] = d[kslot(0, 1, 1)] + kap * (w[kslot(0, 1, 1)] - d[kslot(0, 1, 1)]);
        const float nxx = w[kslot(2, 0, 0)] - d[kslot(2, 0, 0)];
        const float nyy = w[kslot(0, 2, 0)] - d[kslot(0, 2, 0)];
        const float nzz = w[kslot(0, 0, 2)] - d[kslot(0, 0, 2)];
        const float tr = (nxx + nyy + nzz) * (1.0f / 3.0f);
        w[kslot(2, 0, 0)] = d[kslot(2, 0, 0)] + kap * (nxx - tr) + tr;
        w[kslot(0, 2, 0)] = d[kslot(0, 2, 0)] + kap * (nyy - tr) + tr;
        w[kslot(0, 0, 2)] = d[kslot(0, 0, 2)] + kap * (nzz - tr) + tr;
    }

    float uxb = 0.0f, uyb = 0.0f, uzb = 0.0f;
    // scalar: g_out = (1 - kap_s) g^eq(s, u) + kap_s gi
    if (kScalar) {
        const float s = (gi[0] + (gi[1] + gi[2])) + ((gi[3] + gi[4]) + (gi[5] + gi[6]));
        float sb = 0.0f;
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const float me = (1.0f - kap_s) * mu[i];
            const float cu = kSx[i] * ux + kSy[i] * uy + kSz[i] * uz;
            sb += me * kSw[i] * (1.0f + 4.0f * cu);
            const float su = me * kSw[i] * s * 4.0f;
            uxb += su * kSx[i];
            uyb += su * kSy[i];
            uzb += su * kSz[i];
        }
#pragma unroll
        for (int i = 0; i < QS; ++i) gb[i] = kap_s * mu[i] + sb;
    } else {
#pragma unroll
        for (int i = 0; i < QS; ++i) gb[i] = 0.0f;
    }

    // inverse sweeps: out = Ix(Iy(Iz(w)))
    float bar[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) bar[q] = lam[q];
    {
        float t[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) t[q] = w[q];
        sweep_inv<9, 1, 3>(t, uz);
        sweep_inv<3, 1, 9>(t, uy);
        sweep_inv_rev<1, 3, 9>(t, bar, ux, uxb);
#pragma unroll
        for (int q = 0; q < 27; ++q) t[q] = w[q];
        sweep_inv<9, 1, 3>(t, uz);
        sweep_inv_rev<3, 1, 9>(t, bar, uy, uyb);
        sweep_inv_rev<9, 1, 3>(w, bar, uz, uzb);
    }
    // bar = dL/dw; the map: off-diagonal w = d + kap (k - d); diagonal
    // w_a = d_a + kap n_a + (1 - kap) tr with n_a = k_a - d_a, tr = mean n
    float kb[27], db[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        kb[q] = bar[q];
        db[q] = 0.0f;
    }
#define CSLBM_OFFDIAG(m, n, p)                              \
    kb[kslot(m, n, p)] = kap * bar[kslot(m, n, p)];         \
    db[kslot(m, n, p)] = (1.0f - kap) * bar[kslot(m, n, p)];
    CSLBM_OFFDIAG(1, 1, 0)
    CSLBM_OFFDIAG(1, 0, 1)
    CSLBM_OFFDIAG(0, 1, 1)
#undef CSLBM_OFFDIAG
    {
        const float bxx = bar[kslot(2, 0, 0)], byy = bar[kslot(0, 2, 0)], bzz = bar[kslot(0, 0, 2)];
        const float m3 = (1.0f - kap) * (bxx + byy + bzz) * (1.0f / 3.0f);
        const float nxb = kap * bxx + m3, nyb = kap * byy + m3, nzb = kap * bzz + m3;
        kb[kslot(2, 0, 0)] = nxb;
        kb[kslot(0, 2, 0)] = nyb;
        kb[kslot(0, 0, 2)] = nzb;
        db[kslot(2, 0, 0)] = bxx - nxb;
        db[kslot(0, 2, 0)] = byy - nyb;
        db[kslot(0, 0, 2)] = bzz - nzb;
    }
    float drb = 0.0f;
    deviation_equilibrium_rev(db, dr, ux, uy, uz, drb, uxb, uyb, uzb);

    // forward sweeps: k = Fz(Fy(Fx(v)))
    {
        float t[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) t[q] = v[q];
        sweep_fwd<1, 3, 9>(t, ux);
        sweep_fwd<3, 1, 9>(t, uy);
        sweep_fwd_rev<9, 1, 3>(t, kb, uz, uzb);
#pragma unroll
        for (int q = 0; q < 27; ++q) t[q] = v[q];
        sweep_fwd<1, 3, 9>(t, ux);
        sweep_fwd_rev<3, 1, 9>(t, kb, uy, uyb);
        sweep_fwd_rev<1, 3, 9>(v, kb, ux, uxb);
    }
    // u = j ir, dr = sum v, j = sum c v
    const float jxb = uxb * ir, jyb = uyb * ir, jzb = uzb * ir;
    drb += -(uxb * jx + uyb * jy + uzb * jz) * ir * ir;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int cx = t % 3 - 1, cy = (t / 3) % 3 - 1, cz = t / 9 - 1;
        vb[t] = kb[t] + drb + cx * jxb + cy * jyb + cz * jzb;
    }
}

struct ExchAdjArgs {
    ExchArgs e;           // forward exchange (FP32 source states fA, fB)
    float* lam_d;         // dL/d(destination) [27][dplane]: read at the targets, then cleared
    float* mu_d;          // [7][dplane] or null
    float* lam_a;         // dL/d(fA) [27][splane], accumulated
    float* lam_b;         // dL/d(fB), accumulated
    float* mu_a;
    float* mu_b;
    float ca, cb;         // time weights of fA and fB: 1 - w and w (0: not touched)
};

// Adjoint of one exchange launch: one thread per listed target recomputes
// the target's interpolated source state, applies the map's vector-Jacobian
// product to the target's adjoint, clears that adjoint (the forward
// overwrote the target) and adds the trilinear- and time-weighted result to
// the source adjoints of its corners with atomic adds (neighbouring targets
// share corners).
template <bool kScalar, bool kNode>
__global__ void __launch_bounds__(256) k_exchange_adjoint(const ExchAdjArgs a)
{
    const ExchArgs& e = a.e;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= e.n_cells) return;
    const int c = e.cells[k];
    int base[3];
    float t[3];
    target_stencil(e, c, base, t);
    if (kNode) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (t[d] >= 0.5f) ++base[d];
            t[d] = 0.0f;
        }
    }
    const int n[3] = {e.snx, e.sny, e.snz};
    int ix[2], iy[2], iz[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        ix[o] = wrap_or_clamp(base[0] + o, n[0], e.speriodic & 1);
        iy[o] = wrap_or_clamp(base[1] + o, n[1], e.speriodic & 2);
        iz[o] = wrap_or_clamp(base[2] + o, n[2], e.speriodic & 4);
    }
    const float* fA = static_cast<const float*>(e.fA);
    const float* fB = static_cast<const float*>(e.fB);
    const float w = e.w;
    const bool blend = a.ca != 0.0f && a.cb != 0.0f;
    constexpr int kCorners = kNode ? 1 : 8;

    float v[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = 0.0f;
    float gi[QS] = {0, 0, 0, 0, 0, 0, 0};
    for (int corner = 0; corner < kCorners; ++corner) {
        const float wt = corner_weight(t, corner);
        const int64_t sc = ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                              (int64_t)e.sny * iz[(corner >> 2) & 1]);
        for (int i = 0; i < Q; ++i) {
            const float hA = fA[i * e.splane + sc], hB = fB[i * e.splane + sc];
            v[tensor_slot(i)] += wt * (blend ? (1.0f - w) * hA + w * hB : (a.cb != 0.0f ? hB : hA));
        }
        if (kScalar)
            for (int i = 0; i < QS; ++i) {
                const float gA = e.gA[i * e.splane + sc], gB = e.gB[i * e.splane + sc];
                gi[i] += wt * (blend ? (1.0f - w) * gA + w * gB : (a.cb != 0.0f ? gB : gA));
            }
    }
    float lam[27], mu[QS] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        lam[tensor_slot(i)] = a.lam_d[i * e.dplane + c];
        a.lam_d[i * e.dplane + c] = 0.0f;
    }
    if (kScalar)
        for (int i = 0; i < QS; ++i) {
            mu[i] = a.mu_d[i * e.dplane + c];
            a.mu_d[i * e.dplane + c] = 0.0f;
        }
    float vb[27], gb[QS];
    exchange_map_adjoint<kScalar>(v, gi, e.kappa, e.kappa_s, lam, mu, vb, gb);
    for (int corner = 0; corner < kCorners; ++corner) {
        const float wt = corner_weight(t, corner);
        if (wt == 0.0f) continue;
        const int64_t sc = ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                              (int64_t)e.sny * iz[(corner >> 2) & 1]);
        for (int i = 0; i < Q; ++i) {
            const float b = wt * vb[tensor_slot(i)];
            if (a.ca != 0.0f) atomicAdd(a.lam_a + i * e.splane + sc, a.ca * b);
            if (a.cb != 0.0f) atomicAdd(a.lam_b + i * e.splane + sc, a.cb * b);
        }
        if (kScalar)
            for (int i = 0; i < QS; ++i) {
                const float b = wt * gb[i];
                if (a.ca != 0.0f) atomicAdd(a.mu_a + i * e.splane + sc, a.ca * b);
                if (a.cb != 0.0f) atomicAdd(a.mu_b + i * e.splane + sc, a.cb * b);
            }
    }
}

// Gather form of the exchange adjoint, without atomics.  Pass A (one thread
// per target): the target's vector-Jacobian product goes to column k of a
// [34][n] buffer, the target's cell to a dense index map of the destination
// box and its source corners are flagged; targets whose stencil wraps or is
// clamped at the source box's faces are scattered with atomics instead.  Pass
// B (one thread per flagged source cell): the cell sums weight times column
// over the targets whose stencil holds it, found through the index map, and
// adds the sum to its own adjoint entries (one writer per entry).  Pass C
// resets the index map; pass B resets the flags.
struct GatherWs {
    float* vb;          // [34][n_cells] per-target products
    int32_t* map;       // [dst cells]: list index of a gathered target, -1 otherwise
    uint8_t* touched;   // [src cells]: 1 for a source corner of a gathered target
};

// Stencil of list entry k (forward arithmetic): corner indices after wrap or
// clamp, trilinear fractions, and whether the stencil lies inside the source
// box without wrapping or clamping.
template <bool kNode>
__device__ __forceinline__ bool target_corners(const ExchArgs& e, int c, int (&ix)[2], int (&iy)[2],
                                               int (&iz)[2], float (&t)[3])
{
    int base[3];
    target_stencil(e, c, base, t);
    if (kNode) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (t[d] >= 0.5f) ++base[d];
            t[d] = 0.0f;
        }
    }
    const int n[3] = {e.snx, e.sny, e.snz};
    bool interior = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        interior = interior && base[d] >= 0 && base[d] + (kNode ? 0 : 1) <= n[d] - 1;
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        ix[o] = wrap_or_clamp(base[0] + o, n[0], e.speriodic & 1);
        iy[o] = wrap_or_clamp(base[1] + o, n[1], e.speriodic & 2);
        iz[o] = wrap_or_clamp(base[2] + o, n[2], e.speriodic & 4);
    }
    return interior;
}

// Pass A1: the interpolated source state of every target into column k of
// the buffer; index map and corner flags for the gathered targets.
template <bool kScalar, bool kNode, bool kBlend>
__global__ void __launch_bounds__(256) k_exadj_interp(const ExchAdjArgs a, const GatherWs g)
{
    const ExchArgs& e = a.e;
    // without blending the host passes the time level that carries the weight
    const bool use_b = !kBlend && a.cb != 0.0f;
    // the segment of this block (uniform): a staged copy of the parent's
    // columns around one x-face of the shell, or the source level itself
    int blk = blockIdx.x;
    const float* fA = static_cast<const float*>(use_b ? e.fB : e.fA);
    const float* fB = static_cast<const float*>(e.fB);
    const float* gA = use_b ? e.gB : e.gA;
    const float* gB = e.gB;
    int sn[3] = {e.snx, e.sny, e.snz};
    int off[3] = {0, 0, 0};
    int64_t splane = e.splane;
    int first = e.main_first, count = e.n_cells - e.main_first;
    bool staged = false;
#pragma unroll
    for (int sgi = 0; sgi < 2; ++sgi) {
        if (staged || sgi >= e.n_staged) continue;
        if (blk < e.st[sgi].blocks) {
            const ExchArgs::Staged& st = e.st[sgi];
            fA = static_cast<const float*>(use_b ? st.fB : st.fA);
            fB = static_cast<const float*>(st.fB);
            gA = use_b ? st.gB : st.gA;
            gB = st.gB;
            sn[0] = st.nx;
            sn[1] = st.ny;
            sn[2] = st.nz;
            off[0] = st.off[0];
            off[1] = st.off[1];
            off[2] = st.off[2];
            splane = st.plane;
            first = st.first;
            count = st.count;
            staged = true;
        } else {
            blk -= e.st[sgi].blocks;
        }
    }
    const int kl = blk * blockDim.x + threadIdx.x;
    if (kl >= count) return;
    const int k = first + kl;
    const int c = e.cells[k];
    int ix[2], iy[2], iz[2];
    float t[3];
    const bool interior = target_corners<kNode>(e, c, ix, iy, iz, t);
    // corners in the segment's storage (a staged copy holds only its face's
    // stencils: a corner outside it makes the target NaN)
    int lx[2], ly[2], lz[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        lx[o] = ix[o] - off[0];
        ly[o] = iy[o] - off[1];
        lz[o] = iz[o] - off[2];
    }
    const bool outside = staged && (min(lx[0], lx[1]) < 0 || max(lx[0], lx[1]) >= sn[0] || min(ly[0], ly[1]) < 0 ||
                                    max(ly[0], ly[1]) >= sn[1] || min(lz[0], lz[1]) < 0 ||
                                    max(lz[0], lz[1]) >= sn[2]);
    const float w = e.w;
    constexpr int kCorners = kNode ? 1 : 8;
    float v[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = 0.0f;
    float gi[QS] = {0, 0, 0, 0, 0, 0, 0};
    // four corners per pass (two blended: 136 loads in flight either way),
    // summed in order 0..7
    constexpr int kPass = kBlend ? 2 : 4;
#pragma unroll kPass
    for (int corner = 0; corner < kCorners; ++corner) {
        const float wt = corner_weight(t, corner);
        const int64_t sc = outside ? 0
                                   : lx[corner & 1] + (int64_t)sn[0] * (ly[(corner >> 1) & 1] +
                                                                        (int64_t)sn[1] * lz[(corner >> 2) & 1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float hA = fA[i * splane + sc];
            if (kBlend) {
                const float hB = fB[i * splane + sc];
                v[i] += wt * ((1.0f - w) * hA + w * hB);
            } else {
                v[i] += wt * hA;
            }
        }
        if (kScalar)
#pragma unroll
            for (int i = 0; i < QS; ++i) {
                const float g0 = gA[i * splane + sc];
                if (kBlend) {
                    const float g1 = gB[i * splane + sc];
                    gi[i] += wt * ((1.0f - w) * g0 + w * g1);
                } else {
                    gi[i] += wt * g0;
                }
            }
    }
    if (outside) v[13] = __builtin_nanf("");
    const int64_t n_t = e.n_cells;
#pragma unroll
    for (int i = 0; i < Q; ++i) g.vb[i * n_t + k] = v[i];
    if (kScalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) g.vb[(Q + i) * n_t + k] = gi[i];
    if (interior) {
        g.map[c] = k;
#pragma unroll
        for (int corner = 0; corner < kCorners; ++corner)
            g.touched[ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                         (int64_t)e.sny * iz[(corner >> 2) & 1])] = 1;
    }
}

// Pass A2: the map's vector-Jacobian product of every target, from its
// interpolated state (column k) and the target's adjoint (then cleared);
// the result replaces column k, or is scattered with atomics for a target
// outside the gather (stencil wrapped or clamped).
// lam[., c] = 0 and mu[., c] = 0 (the destination adjoint, once read)
template <bool kScalar>
__device__ __forceinline__ void clear_column(float* lam, float* mu, int64_t plane, int c)
{
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[i * plane + c] = 0.0f;
    if (kScalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) mu[i * plane + c] = 0.0f;
}

template <bool kScalar, bool kNode>
__global__ void __launch_bounds__(256) k_exadj_vjp(const ExchAdjArgs a, const GatherWs g)
{
    const ExchArgs& e = a.e;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= e.n_cells) return;
    const int c = e.cells[k];
    const int64_t n_t = e.n_cells;
    float v[27], gi[QS] = {0, 0, 0, 0, 0, 0, 0};
    float lam[27], mu[QS] = {0, 0, 0, 0, 0, 0, 0};
    // every element loaded before the destination adjoint is cleared: all
    // loads in flight together
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        v[tensor_slot(i)] = g.vb[i * n_t + k];
        lam[tensor_slot(i)] = a.lam_d[i * e.dplane + c];
    }
    if (kScalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            gi[i] = g.vb[(Q + i) * n_t + k];
            mu[i] = a.mu_d[i * e.dplane + c];
        }
    clear_column<kScalar>(a.lam_d, a.mu_d, e.dplane, c);
    float vb[27], gb[QS];
    exchange_map_adjoint<kScalar>(v, gi, e.kappa, e.kappa_s, lam, mu, vb, gb);
    // the column addresses are formed again for the stores instead of kept
    // live through the map adjoint (the empty asm hides that kc == k)
    int kc = k;
    asm volatile("" : "+v"(kc));
    if (g.map[c] == kc) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g.vb[i * n_t + kc] = vb[tensor_slot(i)];
        if (kScalar)
#pragma unroll
            for (int i = 0; i < QS; ++i) g.vb[(Q + i) * n_t + kc] = gb[i];
        return;
    }
    int ix[2], iy[2], iz[2];
    float t[3];
    target_corners<kNode>(e, c, ix, iy, iz, t);
    constexpr int kCorners = kNode ? 1 : 8;
    for (int corner = 0; corner < kCorners; ++corner) {
        const float wt = corner_weight(t, corner);
        if (wt == 0.0f) continue;
        const int64_t sc = ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                              (int64_t)e.sny * iz[(corner >> 2) & 1]);
        for (int i = 0; i < Q; ++i) {
            const float b = wt * vb[tensor_slot(i)];
            if (a.ca != 0.0f) atomicAdd(a.lam_a + i * e.splane + sc, a.ca * b);
            if (a.cb != 0.0f) atomicAdd(a.lam_b + i * e.splane + sc, a.cb * b);
        }
        if (kScalar)
            for (int i = 0; i < QS; ++i) {
                const float b = wt * gb[i];
                if (a.ca != 0.0f) atomicAdd(a.mu_a + i * e.splane + sc, a.ca * b);
                if (a.cb != 0.0f) atomicAdd(a.mu_b + i * e.splane + sc, a.cb * b);
            }
    }
}

// Weight of source index s on one axis for destination index j, with the
// forward stencil's arithmetic (target_stencil, then corner_weight's factor).
template <bool kNode>
__device__ __forceinline__ float axis_weight(double dorigin, double ddx, double sorigin, double sdx,
                                             int j, int s)
{
    const double p = dorigin + j * ddx;
    const double q = (p - sorigin) / sdx;
    const double b = floor(q);
    int base = (int)b;
    float t = (float)(q - b);
    if (kNode) {
        if (t >= 0.5f) ++base;
        return base == s ? 1.0f : 0.0f;
    }
    if (base == s) return 1.0f - t;
    if (base + 1 == s) return t;
    return 0.0f;
}

constexpr int kMaxCand = 8;   // destination candidates per axis (host checks the spacing ratio)
constexpr int kList = 3;      // targets collected before their columns are summed (3: fewer loads
                              // in flight, five waves per SIMD; 8 took four)

// sum += weight * column for the collected (k, weight) pairs
template <bool kScalar>
__device__ __forceinline__ void sum_columns(const GatherWs& g, int64_t n_t, const int (&kk)[kList],
                                            const float (&ww)[kList], int nk, float (&acc)[27],
                                            float (&gacc)[QS])
{
#pragma unroll
    for (int e = 0; e < kList; ++e) {
        if (e >= nk) break;
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] += ww[e] * g.vb[i * n_t + kk[e]];
        if (kScalar)
#pragma unroll
            for (int i = 0; i < QS; ++i) gacc[i] += ww[e] * g.vb[(Q + i) * n_t + kk[e]];
    }
}

// lam[., s] += c acc and mu[., s] += c gacc in two halves (planes 0-13 of
// lam, then 14-26 and mu): within a half every element is loaded before the
// first store, so its loads are in flight together (a store between them
// would order each later load after it), and a half keeps few addresses live.
template <int kLo, int kHi>
__device__ __forceinline__ void add_planes(float* p, int64_t plane, int64_t s, float c, const float* acc)
{
    float v[kHi - kLo];
#pragma unroll
    for (int i = kLo; i < kHi; ++i) v[i - kLo] = p[i * plane + s];
#pragma unroll
    for (int i = kLo; i < kHi; ++i) p[i * plane + s] = v[i - kLo] + c * acc[i];
}

template <bool kScalar>
__device__ __forceinline__ void add_column(float* lam, float* mu, int64_t plane, int64_t s, float c,
                                           const float (&acc)[27], const float (&gacc)[QS])
{
    add_planes<0, 14>(lam, plane, s, c, acc);
    if (kScalar) {
        float v[Q - 14], u[QS];
#pragma unroll
        for (int i = 14; i < Q; ++i) v[i - 14] = lam[i * plane + s];
#pragma unroll
        for (int i = 0; i < QS; ++i) u[i] = mu[i * plane + s];
#pragma unroll
        for (int i = 14; i < Q; ++i) lam[i * plane + s] = v[i - 14] + c * acc[i];
#pragma unroll
        for (int i = 0; i < QS; ++i) mu[i * plane + s] = u[i] + c * gacc[i];
    } else {
        add_planes<14, Q>(lam, plane, s, c, acc);
    }
}

// Sub-box of the source level that holds every corner of an interior
// target (the only cells the interpolation pass flags)
struct SrcBox {
    int x0, y0, z0, nx, ny, nz;
};

// Narrow window: the destination spacing exceeds the source spacing (or the
// nodes coincide), so per axis at most two destination indices put weight on
// a source index, found among kNarrowCand candidates.
constexpr int kNarrowCand = 5;   // ceil(2 src dx / dst dx) + 3 <= 5

// The nonzero weights of source index s along one axis over the candidate
// window [lo, hi] (at most kMaxCand indices), in increasing index order; the
// host picks kG at least as large as their count.
template <int kG>
__device__ __forceinline__ int axis_nonzero(double dorigin, double ddx, double sorigin, double sdx, int lo,
                                            int hi, int s, int (&j)[kG], float (&w)[kG])
{
    int n = 0;
#pragma unroll
    for (int m = 0; m < kG; ++m) {
        j[m] = 0;
        w[m] = 0.0f;
    }
#pragma unroll
    for (int c = 0; c < kMaxCand; ++c) {
        const int jc = lo + c;
        const float wc = jc <= hi ? axis_weight<false>(dorigin, ddx, sorigin, sdx, jc, s) : 0.0f;
        if (wc != 0.0f) {
#pragma unroll
            for (int m = 0; m < kG; ++m)
                if (m == n) {
                    j[m] = jc;
                    w[m] = wc;
                }
            ++n;
        }
    }
    return n;
}

template <bool kScalar, bool kNode, int kG>
__global__ void __launch_bounds__(256) k_exadj_sources(const ExchAdjArgs a, const GatherWs g,
                                                       const SrcBox b)
{
    const ExchArgs& e = a.e;
    const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (l >= (int64_t)b.nx * b.ny * b.nz) return;
    const int sxyz[3] = {b.x0 + (int)(l % b.nx), b.y0 + (int)((l / b.nx) % b.ny),
                         b.z0 + (int)(l / ((int64_t)b.nx * b.ny))};
    const int64_t s = sxyz[0] + (int64_t)e.snx * (sxyz[1] + (int64_t)e.sny * sxyz[2]);
    if (!g.touched[s]) return;
    g.touched[s] = 0;
    constexpr bool kNarrow = kG == 2;
    const int nd[3] = {e.dnx, e.dny, e.dnz};
    const double dorg[3] = {e.dorigin[0], e.dorigin[1], e.dorigin[2]};
    const double sorg[3] = {e.sorigin[0], e.sorigin[1], e.sorigin[2]};
    // per axis: destination indices whose stencil can hold source index s,
    // q(j) in [s - 1, s + 1), with one index of margin each side
    int lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double jl = ((sxyz[d] - 1) * e.sdx + sorg[d] - dorg[d]) / e.ddx;
        lo[d] = max(0, (int)floor(jl) - 1);
        hi[d] = min(nd[d] - 1, (int)floor(jl) - 2 + (kNarrow ? kNarrowCand : kMaxCand));
    }
    const int64_t n_t = e.n_cells;
    float acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = 0.0f;
    float gacc[QS] = {0, 0, 0, 0, 0, 0, 0};
    if constexpr (kNarrow) {
        // the (at most two) nonzero weights per axis, in increasing index order
        int jj[3][2];
        float wj[3][2];
        int nj[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            jj[d][0] = jj[d][1] = 0;
            wj[d][0] = wj[d][1] = 0.0f;
            nj[d] = 0;
#pragma unroll
            for (int c = 0; c < kNarrowCand; ++c) {
                const int j = lo[d] + c;
                const float w = j <= hi[d] ? axis_weight<kNode>(dorg[d], e.ddx, sorg[d], e.sdx, j, sxyz[d]) : 0.0f;
                if (w != 0.0f) {
                    if (nj[d] == 0) {
                        jj[d][0] = j;
                        wj[d][0] = w;
                    } else {
                        jj[d][1] = j;
                        wj[d][1] = w;
                    }
                    ++nj[d];
                }
            }
        }
        // more than two (excluded on the host) would drop a target: loud
        if (nj[0] > 2 || nj[1] > 2 || nj[2] > 2) acc[0] = __builtin_nanf("");
        // the index map of all (up to eight) destination cells read at once,
        // then the targets found packed in loop-nest order (z, y, x ascending)
        int km[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ix = c & 1, iy = (c >> 1) & 1, iz = c >> 2;
            const bool ok = ix < nj[0] && iy < nj[1] && iz < nj[2];
            const int k = g.map[ok ? jj[0][ix] + e.dnx * (jj[1][iy] + e.dny * jj[2][iz]) : 0];
            km[c] = ok ? k : -1;
        }
        int kk[8];
        float ww[8];
        int nk = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            kk[c] = 0;
            ww[c] = 0.0f;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (km[c] < 0) continue;
            const float wt = (wj[0][c & 1] * wj[1][(c >> 1) & 1]) * wj[2][c >> 2];
#pragma unroll
            for (int m = 0; m <= c; ++m)
                if (m == nk) {
                    kk[m] = km[c];
                    ww[m] = wt;
                }
            ++nk;
        }
        // columns summed kList targets at a time
#pragma unroll
        for (int base = 0; base < 8; base += kList) {
            if (base >= nk) break;
#pragma unroll
            for (int m = base; m < base + kList && m < 8; ++m) {
                if (m >= nk) break;
#pragma unroll
                for (int i = 0; i < Q; ++i) acc[i] += ww[m] * g.vb[i * n_t + kk[m]];
                if (kScalar)
#pragma unroll
                    for (int i = 0; i < QS; ++i) gacc[i] += ww[m] * g.vb[(Q + i) * n_t + kk[m]];
            }
        }
    } else {
        // wide window (destination spacing at most the source spacing): the
        // (at most kG) nonzero weights along y and x, then per nonzero z
        // plane the index map of its kG x kG destination cells read at once
        int jy[kG], jx[kG];
        float wy[kG], wx[kG];
        const int ny = axis_nonzero<kG>(dorg[1], e.ddx, sorg[1], e.sdx, lo[1], hi[1], sxyz[1], jy, wy);
        const int nx = axis_nonzero<kG>(dorg[0], e.ddx, sorg[0], e.sdx, lo[0], hi[0], sxyz[0], jx, wx);
        if (nx > kG || ny > kG) acc[0] = __builtin_nanf("");   // excluded on the host
        for (int jz = lo[2]; jz <= hi[2]; ++jz) {
            const float wz = axis_weight<false>(dorg[2], e.ddx, sorg[2], e.sdx, jz, sxyz[2]);
            if (wz == 0.0f) continue;
            constexpr int kP = kG * kG;
            int km[kP];
#pragma unroll
            for (int c = 0; c < kP; ++c) {
                const int ix = c % kG, iy = c / kG;
                const bool ok = ix < nx && iy < ny;
                const int k = g.map[ok ? jx[ix] + e.dnx * (jy[iy] + e.dny * jz) : 0];
                km[c] = ok ? k : -1;
            }
            // the targets found, packed in loop-nest order (y, x ascending)
            int kk[kP];
            float ww[kP];
            int nk = 0;
#pragma unroll
            for (int c = 0; c < kP; ++c) {
                kk[c] = 0;
                ww[c] = 0.0f;
            }
#pragma unroll
            for (int c = 0; c < kP; ++c) {
                if (km[c] < 0) continue;
                const float wt = (wx[c % kG] * wy[c / kG]) * wz;
#pragma unroll
                for (int m = 0; m <= c; ++m)
                    if (m == nk) {
                        kk[m] = km[c];
                        ww[m] = wt;
                    }
                ++nk;
            }
            // one target at a time (a uniform index into the packed list)
#pragma unroll 1
            for (int m = 0; m < kP; ++m) {
                if (m >= nk) break;
#pragma unroll
                for (int i = 0; i < Q; ++i) acc[i] += ww[m] * g.vb[i * n_t + kk[m]];
                if (kScalar)
#pragma unroll
                    for (int i = 0; i < QS; ++i) gacc[i] += ww[m] * g.vb[(Q + i) * n_t + kk[m]];
            }
        }
    }
    if (a.ca != 0.0f) add_column<kScalar>(a.lam_a, a.mu_a, e.splane, s, a.ca, acc, gacc);
    if (a.cb != 0.0f) add_column<kScalar>(a.lam_b, a.mu_b, e.splane, s, a.cb, acc, gacc);
}

__global__ void __launch_bounds__(256) k_exadj_reset(int32_t* map, const int32_t* cells, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) map[cells[k]] = -1;
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill_value(T* p, int64_t n, T value)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// y = alpha x + beta y over n elements
__global__ void __launch_bounds__(256) k_axpby(const float* x, float* y, int64_t n, float alpha,
                                               float beta)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = alpha * x[i] + beta * y[i];
}

// two such updates from one x: y = a1 x + b1 y and z = a2 x + b2 z (x read once)
__global__ void __launch_bounds__(256) k_axpby2(const float* x, float* y, float* z, int64_t n, float a1,
                                                float b1, float a2, float b2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float xi = x[i];
    y[i] = a1 * xi + b1 * y[i];
    z[i] = a2 * xi + b2 * z[i];
}

// z = x + y over n elements
__global__ void __launch_bounds__(256) k_sum(const float* x, const float* y, float* z, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) z[i] = x[i] + y[i];
}

__global__ void __launch_bounds__(256) k_zero(float* p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Pass A2 of one target whose interpolated state (v in tensor order, gi)
// is in registers: the map's vector-Jacobian product into column k (index
// map and corner flags as pass A1 sets them), or scattered with atomics for
// a target outside the gather, as pass A2 does (k_exadj_tiled keeps its own
// copy of these steps: through this function the compiler gave it 278
// VGPRs instead of 182).
template <bool kScalar, bool kNode>
__device__ __forceinline__ void vjp_in_registers(const ExchAdjArgs& a, const GatherWs& g, int k, int c,
                                                 const float (&v)[27], const float (&gi)[QS])
{
    const ExchArgs& e = a.e;
    constexpr int kCorners = kNode ? 1 : 8;
    float lam[27], mu[QS] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[tensor_slot(i)] = a.lam_d[i * e.dplane + c];
    if (kScalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) mu[i] = a.mu_d[i * e.dplane + c];
    clear_column<kScalar>(a.lam_d, a.mu_d, e.dplane, c);
    float vb[27], gb[QS];
    exchange_map_adjoint<kScalar>(v, gi, e.kappa, e.kappa_s, lam, mu, vb, gb);
    int ix[2], iy[2], iz[2];
    float t[3];
    const bool interior = target_corners<kNode>(e, c, ix, iy, iz, t);
    if (interior) {
        const int64_t n_t = e.n_cells;
#pragma unroll
        for (int i = 0; i < Q; ++i) g.vb[i * n_t + k] = vb[tensor_slot(i)];
        if (kScalar)
#pragma unroll
            for (int i = 0; i < QS; ++i) g.vb[(Q + i) * n_t + k] = gb[i];
        g.map[c] = k;
#pragma unroll
        for (int corner = 0; corner < kCorners; ++corner)
            g.touched[ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                         (int64_t)e.sny * iz[(corner >> 2) & 1])] = 1;
        return;
    }
    for (int corner = 0; corner < kCorners; ++corner) {
        const float wt = corner_weight(t, corner);
        if (wt == 0.0f) continue;
        const int64_t sc = ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                              (int64_t)e.sny * iz[(corner >> 2) & 1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float b = wt * vb[tensor_slot(i)];
            if (a.ca != 0.0f) atomicAdd(a.lam_a + i * e.splane + sc, a.ca * b);
            if (a.cb != 0.0f) atomicAdd(a.lam_b + i * e.splane + sc, a.cb * b);
        }
        if (kScalar)
#pragma unroll
            for (int i = 0; i < QS; ++i) {
                const float b = wt * gb[i];
                if (a.ca != 0.0f) atomicAdd(a.mu_a + i * e.splane + sc, a.ca * b);
                if (a.cb != 0.0f) atomicAdd(a.mu_b + i * e.splane + sc, a.cb * b);
            }
    }
}

// Passes A1 and A2 in one for a post-mapping list in tile runs (tile.hpp):
// the run's source box is staged through LDS, every target's interpolated
// state stays in registers, the map's vector-Jacobian product follows, and
// only its result is written to column k.  The index map and corner flags
// are set as pass A1 sets them, and a target outside the gather is
// scattered with atomics as pass A2 scatters it, so the source pass reads
// the same columns bit for bit.  e.fA / e.gA hold the time level that
// carries the weight.  kShell: patch runs of a ghost shell (small boxes, the
// x-plane runs from the staged copies, both time levels blended with
// kBlend), as the forward prior-mapping takes them.
template <bool kScalar, bool kShell = false, bool kBlend = false>
__global__ void __launch_bounds__(256) k_exadj_tiled(const ExchAdjArgs a, const GatherWs g,
                                                     const int32_t* runs)
{
    const ExchArgs& e = a.e;
    TileTarget T;
    float v[27], gi[QS];
    if constexpr (kShell) {
        __shared__ ShellLds lds;
        if (!tile_interp<float, kScalar, kBlend, kShellLoads, kShellPlanes, true>(e, runs, lds, T, v, gi))
            return;
    } else {
        __shared__ TileLds lds;
        if (!tile_interp<float, kScalar>(e, runs, lds, T, v, gi)) return;
    }
    if (!T.active) return;
    const int c = T.c;
    float lam[27], mu[QS] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[tensor_slot(i)] = a.lam_d[i * e.dplane + c];
    if (kScalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) mu[i] = a.mu_d[i * e.dplane + c];
    clear_column<kScalar>(a.lam_d, a.mu_d, e.dplane, c);
    float vb[27], gb[QS];
    exchange_map_adjoint<kScalar>(v, gi, e.kappa, e.kappa_s, lam, mu, vb, gb);
    int ix[2], iy[2], iz[2];
    float t[3];
    const bool interior = target_corners<false>(e, c, ix, iy, iz, t);
    if (interior) {
        const int64_t n_t = e.n_cells;
        const int k = T.k;
#pragma unroll
        for (int i = 0; i < Q; ++i) g.vb[i * n_t + k] = vb[tensor_slot(i)];
        if (kScalar)
#pragma unroll
            for (int i = 0; i < QS; ++i) g.vb[(Q + i) * n_t + k] = gb[i];
        g.map[c] = k;
#pragma unroll
        for (int corner = 0; corner < 8; ++corner)
            g.touched[ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                         (int64_t)e.sny * iz[(corner >> 2) & 1])] = 1;
        return;
    }
    for (int corner = 0; corner < 8; ++corner) {
        const float wt = corner_weight(t, corner);
        if (wt == 0.0f) continue;
        const int64_t sc = ix[corner & 1] + (int64_t)e.snx * (iy[(corner >> 1) & 1] +
                                                              (int64_t)e.sny * iz[(corner >> 2) & 1]);
        for (int i = 0; i < Q; ++i) {
            const float b = wt * vb[tensor_slot(i)];
            if (a.ca != 0.0f) atomicAdd(a.lam_a + i * e.splane + sc, a.ca * b);
            if (a.cb != 0.0f) atomicAdd(a.lam_b + i * e.splane + sc, a.cb * b);
        }
        if (kScalar)
            for (int i = 0; i < QS; ++i) {
                const float b = wt * gb[i];
                if (a.ca != 0.0f) atomicAdd(a.mu_a + i * e.splane + sc, a.ca * b);
                if (a.cb != 0.0f) atomicAdd(a.mu_b + i * e.splane + sc, a.cb * b);
            }
    }
}

// Passes A1 and A2 in one for a list whose targets are all source lattice
// points (one corner of weight 1 each) at one time level: e.fA / e.gA hold
// the level that carries the weight.  The interpolated state is formed as
// pass A1 forms it and kept in registers.
template <bool kScalar>
__global__ void __launch_bounds__(256) k_exadj_node(const ExchAdjArgs a, const GatherWs g)
{
    const ExchArgs& e = a.e;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= e.n_cells) return;
    const int c = e.cells[k];
    int ix[2], iy[2], iz[2];
    float t[3];
    target_corners<true>(e, c, ix, iy, iz, t);
    const float wt = corner_weight(t, 0);
    const int64_t sc = ix[0] + (int64_t)e.snx * (iy[0] + (int64_t)e.sny * iz[0]);
    const float* fA = static_cast<const float*>(e.fA);
    float v[27], gi[QS] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = 0.0f;
#pragma unroll
    for (int i = 0; i < Q; ++i) v[tensor_slot(i)] += wt * fA[i * e.splane + sc];
    if (kScalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) gi[i] += wt * e.gA[i * e.splane + sc];
    vjp_in_registers<kScalar, true>(a, g, k, c, v, gi);
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// The source indices an interior target's stencil can reach: the targets lie
// in dst's box, so per axis floor(q) .. floor(q) + 1 over the box's extent in
// source coordinates q, with one index of margin each side for rounding,
// clipped to the source box (corners of interior targets never wrap).
static SrcBox source_box(const cslbm_level* src, const cslbm_level* dst)
{
    const int sn[3] = {src->nx, src->ny, src->nz}, dn[3] = {dst->nx, dst->ny, dst->nz};
    int lo[3], cnt[3];
    for (int d = 0; d < 3; ++d) {
        const double q0 = (dst->origin[d] - src->origin[d]) / src->dx;
        const double q1 = (dst->origin[d] + (dn[d] - 1) * dst->dx - src->origin[d]) / src->dx;
        const double qa = std::floor(std::min(q0, q1)), qb = std::floor(std::max(q0, q1));
        const double l = std::max(0.0, qa - 1.0), h = std::min((double)(sn[d] - 1), qb + 2.0);
        lo[d] = (int)l;
        cnt[d] = h >= l ? (int)(h - l) + 1 : 0;
    }
    return SrcBox{lo[0], lo[1], lo[2], cnt[0], cnt[1], cnt[2]};
}

// Every corner of every target lies in source_box(src, dst) unless a
// stencil can wrap around a periodic axis of src (the dst box then comes
// within one cell of that axis' ends).
static bool source_box_holds_stencils(const cslbm_level* src, const cslbm_level* dst)
{
    const int sn[3] = {src->nx, src->ny, src->nz}, dn[3] = {dst->nx, dst->ny, dst->nz};
    for (int d = 0; d < 3; ++d) {
        if (!((src->periodic >> d) & 1)) continue;
        const double q0 = (dst->origin[d] - src->origin[d]) / src->dx;
        const double q1 = (dst->origin[d] + (dn[d] - 1) * dst->dx - src->origin[d]) / src->dx;
        if (std::floor(std::min(q0, q1)) < 0.0 || std::floor(std::max(q0, q1)) + 1.0 > sn[d] - 1) return false;
    }
    return true;
}

// z = 0 over the cells of box b of an nx x ny level, all `planes` planes of
// `plane` elements: one thread per box cell (boxes are validated below 2^31
// cells)
__global__ void __launch_bounds__(256) k_box_zero(float* z, int planes, int64_t plane, int nx, int ny,
                                                  const SrcBox b)
{
    const unsigned r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (unsigned)b.nx * b.ny * b.nz) return;
    const unsigned bxy = (unsigned)b.nx * b.ny;
    const int cx = b.x0 + (int)(r % b.nx), cy = b.y0 + (int)((r / b.nx) % b.ny), cz = b.z0 + (int)(r / bxy);
    const int64_t c = cx + (int64_t)nx * (cy + (int64_t)ny * cz);
    for (int pl = 0; pl < planes; ++pl) z[pl * plane + c] = 0.0f;
}

// z = x, plus y over the cells of box b, for the kPlanes planes of every
// cell of an nx x ny x nz level (one thread per cell, grid of the step
// kernels; all loads before the first store)
template <int kPlanes>
__global__ void __launch_bounds__(256) k_copy_add_box(const float* x, const float* y, float* z, int64_t plane,
                                                      int nx, int ny, const SrcBox b)
{
    const int cx = blockIdx.x * blockDim.x + threadIdx.x;
    const int cy = blockIdx.y * blockDim.y + threadIdx.y;
    const int cz = blockIdx.z;
    if (cx >= nx || cy >= ny) return;
    const int64_t c = cx + (int64_t)nx * (cy + (int64_t)ny * cz);
    const bool in_box = (unsigned)(cx - b.x0) < (unsigned)b.nx && (unsigned)(cy - b.y0) < (unsigned)b.ny &&
                        (unsigned)(cz - b.z0) < (unsigned)b.nz;
    float v[kPlanes];
#pragma unroll
    for (int i = 0; i < kPlanes; ++i) v[i] = x[i * plane + c];
    if (in_box) {
        float u[kPlanes];
#pragma unroll
        for (int i = 0; i < kPlanes; ++i) u[i] = y[i * plane + c];
#pragma unroll
        for (int i = 0; i < kPlanes; ++i) v[i] += u[i];
    }
#pragma unroll
    for (int i = 0; i < kPlanes; ++i) z[i * plane + c] = v[i];
}

// Most destination points with a nonzero weight on one source index along an
// axis, for destination spacing r (in source cells, r <= 1).  The weights are
// nonzero for q in (s - 1, s + 1 - 2^-25) (q the destination point in source
// units; the upper end is where the FP32 fraction rounds to 1), so n points
// need (n - 1) r' < 2 - 2^-25, r' the spacing of the computed q, within 1e-9
// of r.
static int max_nonzero_per_axis(double r)
{
    const double x = (2.0 - std::ldexp(1.0, -25)) / (r - 1e-9);
    return (int)std::ceil(x);
}

// source pass with kG nonzero destination weights per axis at most (2:
// narrow window over all three axes at once; 3, 4: per z plane)
template <bool kScalar, bool kNode>
static void launch_sources(const ExchAdjArgs& a, const GatherWs& g, const SrcBox& sb, int kg, dim3 sgrid,
                           hipStream_t stream)
{
    const dim3 block(256);
    if (kg <= 2)
        hipLaunchKernelGGL((k_exadj_sources<kScalar, kNode, 2>), sgrid, block, 0, stream, a, g, sb);
    else if (kNode)
        return;   // coincident nodes always take the narrow window
    else if (kg == 3)
        hipLaunchKernelGGL((k_exadj_sources<kScalar, false, 3>), sgrid, block, 0, stream, a, g, sb);
    else
        hipLaunchKernelGGL((k_exadj_sources<kScalar, false, 4>), sgrid, block, 0, stream, a, g, sb);
}

// Whether scale i's x-face stage overlaps another scale's (a caller may let
// scales share one): then the recompute's copy for scale i may be gone.
static bool stage_shared(const cslbm_scale* S, int ns, int i)
{
    if (!S[i].stage) return false;
    const char* a0 = static_cast<const char*>(S[i].stage);
    const char* a1 = a0 + S[i].stage_bytes;
    for (int j = 0; j < ns; ++j) {
        if (j == i || !S[j].stage) continue;
        const char* b0 = static_cast<const char*>(S[j].stage);
        const char* b1 = b0 + S[j].stage_bytes;
        if (a0 < b1 && b0 < a1) return true;
    }
    return false;
}

// adjoint of launch_exchange(src, fA, fB, w, dst, ..., cells): the
// destination adjoint lam_d (mu_d) at the cells goes to the source adjoints
static int launch_exchange_adjoint(const cslbm_level* src, const void* fA, const void* fB,
                                   const float* gA, const float* gB, double w,
                                   const cslbm_level* dst, float* lam_d, float* mu_d,
                                   float* lam_a, float* lam_b, float* mu_a, float* mu_b,
                                   const int32_t* cells, int32_t n_cells, const GatherWs* gw,
                                   hipStream_t stream, const int32_t* runs = nullptr,
                                   int32_t n_runs = 0, const cslbm_scale* stage_sc = nullptr,
                                   bool staged = false, bool shell = false)
{
    if (n_cells == 0) return CSLBM_OK;
    const bool scalar = gA != nullptr && mu_d != nullptr;
    ExchAdjArgs a;
    a.e = exchange_args(src, fA, fB, scalar ? gA : nullptr, scalar ? gB : nullptr, w, dst, nullptr,
                        scalar ? mu_d : nullptr, cells, n_cells);
    // a prior-mapping of stage_sc's shell whose x-face entries the forward
    // step read from the staged copies: the interpolation pass reads them
    // there too (the same values, contiguous)
    if (stage_sc) prior_segments(*stage_sc, staged, src, a.e);
    a.lam_d = lam_d;
    a.mu_d = scalar ? mu_d : nullptr;
    a.lam_a = lam_a;
    a.lam_b = lam_b;
    a.mu_a = mu_a;
    a.mu_b = mu_b;
    a.ca = w >= 1.0 ? 0.0f : (float)(1.0 - w);
    a.cb = w <= 0.0 ? 0.0f : (float)w;
    const dim3 grid(grid_for(n_cells)), block(256);
    // The candidate window of the gather pass spans q(j) in [s - 1, s + 1)
    // plus one index each side: 2 src->dx / dst->dx + 4 indices at most.
    // Per axis the nonzero weights of a source index belong to the
    // destination points q in (s - 1, s + 1) (source units; nodes:
    // [s - 1/2, s + 1/2)), spaced r = dst dx / src dx apart: at most two for
    // r > 1 or nodes, else max_nonzero_per_axis(r) (4 for r = 1/2).
    const double r = dst->dx / src->dx;
    const bool node = nodes_coincide(src, dst);
    const int kg = (node || r > 1.0 + 1e-6) ? 2 : max_nonzero_per_axis(r);
    if (gw && 2.0 * src->dx / dst->dx + 4.0 <= (double)kMaxCand && kg <= 4) {
        const GatherWs g = *gw;
        const SrcBox sb = source_box(src, dst);
        const int64_t n_box = (int64_t)sb.nx * sb.ny * sb.nz;
        const dim3 sgrid(grid_for(n_box > 0 ? n_box : 1));
        const bool blend = a.ca != 0.0f && a.cb != 0.0f;
        if (runs && n_runs > 0 && (shell || !blend) && !node && a.e.speriodic == 0 && !a.e.sb.table &&
            !a.e.db.table) {
            // passes A1 and A2 fused, one workgroup per run
            ExchAdjArgs t = a;
            if (a.ca == 0.0f) {
                t.e.fA = t.e.fB;
                t.e.gA = t.e.gB;
                for (int sgi = 0; sgi < t.e.n_staged; ++sgi) {
                    t.e.st[sgi].fA = t.e.st[sgi].fB;
                    t.e.st[sgi].gA = t.e.st[sgi].gB;
                }
            }
            const dim3 rgrid((unsigned)n_runs);
            if (shell && blend) {
                if (scalar)
                    hipLaunchKernelGGL((k_exadj_tiled<true, true, true>), rgrid, block, 0, stream, t, g, runs);
                else
                    hipLaunchKernelGGL((k_exadj_tiled<false, true, true>), rgrid, block, 0, stream, t, g, runs);
            } else if (shell) {
                if (scalar)
                    hipLaunchKernelGGL((k_exadj_tiled<true, true, false>), rgrid, block, 0, stream, t, g, runs);
                else
                    hipLaunchKernelGGL((k_exadj_tiled<false, true, false>), rgrid, block, 0, stream, t, g, runs);
            } else if (scalar) {
                hipLaunchKernelGGL(k_exadj_tiled<true>, rgrid, block, 0, stream, t, g, runs);
            } else {
                hipLaunchKernelGGL(k_exadj_tiled<false>, rgrid, block, 0, stream, t, g, runs);
            }
            if (scalar)
                launch_sources<true, false>(a, g, sb, kg, sgrid, stream);
            else
                launch_sources<false, false>(a, g, sb, kg, sgrid, stream);
            hipLaunchKernelGGL(k_exadj_reset, grid, block, 0, stream, g.map, cells, n_cells);
            return check_launch("k_exchange_adjoint (tiled gather)");
        }
        if (node && !blend && a.e.n_staged == 0) {
            // passes A1 and A2 fused, one thread per target
            ExchAdjArgs t = a;
            if (a.ca == 0.0f) {
                t.e.fA = t.e.fB;
                t.e.gA = t.e.gB;
            }
            if (scalar) {
                hipLaunchKernelGGL(k_exadj_node<true>, grid, block, 0, stream, t, g);
                launch_sources<true, true>(a, g, sb, kg, sgrid, stream);
            } else {
                hipLaunchKernelGGL(k_exadj_node<false>, grid, block, 0, stream, t, g);
                launch_sources<false, true>(a, g, sb, kg, sgrid, stream);
            }
            hipLaunchKernelGGL(k_exadj_reset, grid, block, 0, stream, g.map, cells, n_cells);
            return check_launch("k_exchange_adjoint (node gather)");
        }
        // the interpolation pass runs the staged segments' blocks first
        int64_t iblocks = (n_cells - a.e.main_first + 255) / 256;
        for (int sgi = 0; sgi < a.e.n_staged; ++sgi) iblocks += a.e.st[sgi].blocks;
        const dim3 igrid((unsigned)iblocks);
#define CSLBM_GATHER(S_, N_)                                                                   \
        if (blend)                                                                             \
            hipLaunchKernelGGL((k_exadj_interp<S_, N_, true>), igrid, block, 0, stream, a, g); \
        else                                                                                   \
            hipLaunchKernelGGL((k_exadj_interp<S_, N_, false>), igrid, block, 0, stream, a, g); \
        hipLaunchKernelGGL((k_exadj_vjp<S_, N_>), grid, block, 0, stream, a, g);              \
        launch_sources<S_, N_>(a, g, sb, kg, sgrid, stream);
        if (scalar && node) {
            CSLBM_GATHER(true, true)
        } else if (scalar) {
            CSLBM_GATHER(true, false)
        } else if (node) {
            CSLBM_GATHER(false, true)
        } else {
            CSLBM_GATHER(false, false)
        }
#undef CSLBM_GATHER
        hipLaunchKernelGGL(k_exadj_reset, grid, block, 0, stream, g.map, cells, n_cells);
        return check_launch("k_exchange_adjoint (gather)");
    }
    if (scalar) {
        if (node)
            hipLaunchKernelGGL((k_exchange_adjoint<true, true>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((k_exchange_adjoint<true, false>), grid, block, 0, stream, a);
    } else {
        if (node)
            hipLaunchKernelGGL((k_exchange_adjoint<false, true>), grid, block, 0, stream, a);
        else
            hipLaunchKernelGGL((k_exchange_adjoint<false, false>), grid, block, 0, stream, a);
    }
    return check_launch("k_exchange_adjoint");
}

// Sub-step schedule of a finer scale (Algorithm 1 with the quadratic time
// interpolation through 0, (l-1)/alpha, l/alpha evaluated at 1).
struct SubSteps {
    double alpha, l0, l1, l2;
    int l, last;
    bool node;   // integer alpha: the last sub-step has weight 0 and is skipped
};

static SubSteps sub_steps(const cslbm_scale* S, int i)
{
    SubSteps s;
    s.alpha = S[0].level.dx / S[i].level.dx;
    s.l = (int)std::floor(s.alpha + 1e-12) + 1;
    const double t0 = 0.0, t1 = (s.l - 1) / s.alpha, t2 = s.l / s.alpha;
    s.l0 = (1.0 - t1) * (1.0 - t2) / ((t0 - t1) * (t0 - t2));
    s.l1 = (1.0 - t0) * (1.0 - t2) / ((t1 - t0) * (t1 - t2));
    s.l2 = (1.0 - t0) * (1.0 - t1) / ((t2 - t0) * (t2 - t1));
    s.node = s.l2 == 0.0 && s.l0 == 0.0 && s.l1 == 1.0;
    s.last = s.node ? s.l - 1 : s.l;
    return s;
}

// A population state (27 planes) with its scalar (7 planes) in the workspace.
struct Buf {
    float* f;
    float* g;
};

struct Layout {
    int64_t bytes;
    Buf B0;                          // reference scale after its step
    Buf cur[CSLBM_MAX_SCALES][8];    // inputs of the sub-steps 2..last (index k - 1)
    Buf R[CSLBM_MAX_SCALES];         // interpolated state of a finer scale
    Buf lamA[CSLBM_MAX_SCALES];      // adjoint of each scale's state after its first prior-map
    Buf t1[CSLBM_MAX_SCALES], t2[CSLBM_MAX_SCALES];   // adjoint temporaries
    GatherWs gather;                 // gather form of the exchange adjoints
    int64_t max_cells;               // largest scale (index map and flags)
};

static int64_t gather_bytes(int64_t n_targets, int64_t dst_cells, int64_t src_cells)
{
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    return up((int64_t)(Q + QS) * n_targets * 4) + up(dst_cells * 4) + up(src_cells);
}

static GatherWs gather_at(char* base, int64_t n_targets, int64_t dst_cells)
{
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    GatherWs g;
    g.vb = reinterpret_cast<float*>(base);
    g.map = reinterpret_cast<int32_t*>(base + up((int64_t)(Q + QS) * n_targets * 4));
    g.touched = reinterpret_cast<uint8_t*>(base + up((int64_t)(Q + QS) * n_targets * 4) + up(dst_cells * 4));
    return g;
}

static int64_t buf_bytes(const cslbm_level* L, bool scalar)
{
    const int64_t b = ((int64_t)Q + (scalar ? QS : 0)) * L->plane * 4;
    return (b + 255) / 256 * 256;
}

// Workspace layout; with base == nullptr only the size is computed.
static Layout layout(const cslbm_hierarchy* H, char* base)
{
    Layout o;
    std::memset(&o, 0, sizeof o);
    const cslbm_scale* S = H->scales;
    const bool scalar = S[0].level.g != nullptr;
    int64_t off = 0;
    auto take = [&](const cslbm_level* L) {
        Buf b;
        b.f = base ? reinterpret_cast<float*>(base + off) : nullptr;
        b.g = (base && scalar) ? b.f + (int64_t)Q * L->plane : nullptr;
        off += buf_bytes(L, scalar);
        return b;
    };
    o.B0 = take(&S[0].level);
    o.lamA[0] = take(&S[0].level);
    o.t1[0] = take(&S[0].level);
    for (int i = 1; i < H->n_scales; ++i) {
        const SubSteps ss = sub_steps(S, i);
        for (int k = 1; k < ss.last; ++k) o.cur[i][k] = take(&S[i].level);   // k = 0: f_in[i]
        o.R[i] = take(&S[i].level);
        o.lamA[i] = take(&S[i].level);
        o.t1[i] = take(&S[i].level);
        o.t2[i] = take(&S[i].level);
    }
    int64_t max_targets = 0, max_cells = 0;
    for (int i = 0; i < H->n_scales; ++i) {
        const cslbm_level* L = &S[i].level;
        max_cells = std::max<int64_t>(max_cells, (int64_t)L->nx * L->ny * L->nz);
        if (i == 0) continue;
        max_targets = std::max<int64_t>(max_targets, S[i].n_ghost);
        for (int j = 0; j < i; ++j) max_targets = std::max<int64_t>(max_targets, S[i].n_post[j]);
    }
    o.max_cells = max_cells;
    o.gather = base ? gather_at(base + off, max_targets, max_cells) : GatherWs{nullptr, nullptr, nullptr};
    off += gather_bytes(max_targets, max_cells, max_cells);
    o.bytes = off;
    return o;
}

static int validate_adjoint_hierarchy(const cslbm_hierarchy* H)
{
    int rc = validate_hierarchy(H);
    if (rc) return rc;
    const cslbm_scale* S = H->scales;
    for (int i = 0; i < H->n_scales; ++i) {
        const cslbm_level* L = &S[i].level;
        if (L->storage != CSLBM_F32)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: the multi-scale adjoint needs FP32 storage", i);
        if (L->brick_table)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: brick levels are not differentiated", i);
        if (L->wall_cells != 0)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: wall nodes are not differentiated", i);
        if (i > 0 && L->dx > S[0].level.dx)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: far-field scales are not differentiated", i);
        if (i > 0 && S[i].parent != i - 1)
            return fail(CSLBM_ERR_UNSUPPORTED,
                        "scale %d: the multi-scale adjoint needs a chain (parent of scale i is i - 1)", i);
        if (!L->flags && (L->periodic & 7) != 7)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: a level without flags must be periodic", i);
        if (i > 0 && sub_steps(S, i).last > 8)
            return fail(CSLBM_ERR_UNSUPPORTED, "scale %d: more than 8 sub-steps", i);
    }
    return CSLBM_OK;
}

static void axpby(const float* x, float* y, int64_t n, float alpha, float beta, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, x, y, n, alpha, beta);
}

}  // namespace cslbm

using namespace cslbm;

extern "C" {

int64_t cslbm_exchange_adjoint_bytes(const cslbm_level* src, const cslbm_level* dst, int32_t n_cells)
{
    if (!src || !dst || n_cells < 0) return -1;
    return gather_bytes(n_cells, (int64_t)dst->nx * dst->ny * dst->nz,
                        (int64_t)src->nx * src->ny * src->nz);
}

int cslbm_exchange_adjoint(const cslbm_level* src, const void* fA, const void* fB, const float* gA,
                           const float* gB, double w, const cslbm_level* dst, float* lam_d,
                           float* mu_d, float* lam_a, float* lam_b, float* mu_a, float* mu_b,
                           const int32_t* cells, int32_t n_cells, void* workspace,
                           int64_t workspace_bytes, hipStream_t stream)
{
    int rc = validate_shape(src);
    if (rc) return rc;
    rc = validate_shape(dst);
    if (rc) return rc;
    if (src->storage != CSLBM_F32)
        return fail(CSLBM_ERR_UNSUPPORTED, "the exchange adjoint reads FP32 source states");
    if (src->brick_table || dst->brick_table)
        return fail(CSLBM_ERR_UNSUPPORTED, "the exchange adjoint of brick levels");
    if (src->wall_cells != 0 || dst->wall_cells != 0)
        return fail(CSLBM_ERR_UNSUPPORTED, "the exchange adjoint of levels with wall nodes");
    if (!(src->dx > 0.0) || !(dst->dx > 0.0)) return fail(CSLBM_ERR_ARG, "scale spacings must be positive");
    if (std::fabs(1.0 - shear_rate(src)) < 1e-9)
        return fail(CSLBM_ERR_ARG, "source relaxation time is 1: the mapping is singular");
    if (!(w >= 0.0 && w <= 1.0)) return fail(CSLBM_ERR_ARG, "time weight %g outside [0, 1]", w);
    if (n_cells < 0 || (n_cells > 0 && !cells)) return fail(CSLBM_ERR_ARG, "bad cell list");
    if (!fA || !lam_d) return fail(CSLBM_ERR_ARG, "source state or destination adjoint is NULL");
    if ((w < 1.0 && !lam_a) || (w > 0.0 && (!fB || !lam_b)))
        return fail(CSLBM_ERR_ARG, "a time level with nonzero weight needs its state and adjoint");
    const bool scalar = gA && mu_d;
    if (scalar && ((w < 1.0 && !mu_a) || (w > 0.0 && (!gB || !mu_b))))
        return fail(CSLBM_ERR_ARG, "scalar adjoint buffers are NULL");
    if (lam_d == lam_a || lam_d == lam_b) return fail(CSLBM_ERR_ARG, "destination and source adjoints alias");
    if (w > 0.0 && w < 1.0 && lam_a == lam_b)
        return fail(CSLBM_ERR_ARG, "the two time levels' adjoints alias");
    GatherWs g{nullptr, nullptr, nullptr};
    if (workspace) {
        const int64_t need = cslbm_exchange_adjoint_bytes(src, dst, n_cells);
        if (workspace_bytes < need)
            return fail(CSLBM_ERR_ARG, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes,
                        (long long)need);
        const int64_t nd = (int64_t)dst->nx * dst->ny * dst->nz, ns = (int64_t)src->nx * src->ny * src->nz;
        g = gather_at(static_cast<char*>(workspace), n_cells, nd);
        hipLaunchKernelGGL(k_fill_value<int32_t>, dim3(grid_for(nd)), dim3(256), 0, stream, g.map, nd, -1);
        hipLaunchKernelGGL(k_fill_value<uint8_t>, dim3(grid_for(ns)), dim3(256), 0, stream, g.touched, ns,
                           (uint8_t)0);
    }
    return launch_exchange_adjoint(src, fA, fB ? fB : fA, scalar ? gA : nullptr,
                                   scalar ? (gB ? gB : gA) : nullptr, w, dst, lam_d,
                                   scalar ? mu_d : nullptr, lam_a, lam_b, mu_a, mu_b, cells, n_cells,
                                   workspace ? &g : nullptr, stream);
}

int64_t cslbm_multiscale_adjoint_bytes(const cslbm_hierarchy* H)
{
    if (validate_adjoint_hierarchy(H)) return -1;
    return layout(H, nullptr).bytes;
}

int cslbm_multiscale_adjoint_step(const cslbm_hierarchy* H, const void* const* f_in,
                                  const float* const* g_in, float* const* lam, float* const* mu,
                                  void* workspace, int64_t workspace_bytes, hipStream_t stream)
{
    int rc = validate_adjoint_hierarchy(H);
    if (rc) return rc;
    const int ns = H->n_scales;
    const cslbm_scale* S = H->scales;
    const bool scalar = S[0].level.g != nullptr;
    if (!f_in || !lam) return fail(CSLBM_ERR_ARG, "state or adjoint arrays are NULL");
    if (scalar && (!g_in || !mu)) return fail(CSLBM_ERR_ARG, "scalar state or adjoint arrays are NULL");
    for (int i = 0; i < ns; ++i) {
        if (!f_in[i] || !lam[i]) return fail(CSLBM_ERR_ARG, "scale %d: NULL state or adjoint", i);
        if (scalar && (!g_in[i] || !mu[i]))
            return fail(CSLBM_ERR_ARG, "scale %d: NULL scalar state or adjoint", i);
    }
    const Layout need = layout(H, nullptr);
    if (!workspace || workspace_bytes < need.bytes)
        return fail(CSLBM_ERR_ARG, "workspace of %lld bytes, %lld needed", (long long)workspace_bytes,
                    (long long)need.bytes);
    Layout W = layout(H, static_cast<char*>(workspace));
    auto nelem = [&](int i) { return ((int64_t)Q + (scalar ? QS : 0)) * S[i].level.plane; };

    // ---- forward recompute of the reference step from the states at t_n ----
    bool stage_used[CSLBM_MAX_SCALES] = {};
    const void* A[CSLBM_MAX_SCALES];
    const void* B[CSLBM_MAX_SCALES];
    const float* gA[CSLBM_MAX_SCALES];
    const float* gB[CSLBM_MAX_SCALES];
    {
        const cslbm_level* L = &S[0].level;
        rc = launch_step_into(L, f_in[0], W.B0.f, scalar ? g_in[0] : nullptr, W.B0.g, stream);
        if (rc) return rc;
        A[0] = f_in[0];
        gA[0] = scalar ? g_in[0] : nullptr;
        B[0] = W.B0.f;
        gB[0] = W.B0.g;
    }
    for (int i = 1; i < ns; ++i) {
        const cslbm_scale& sc = S[i];
        const cslbm_level* L = &sc.level;
        const cslbm_level* P = &S[i - 1].level;
        const int p = i - 1;
        const SubSteps ss = sub_steps(S, i);
        // the first sub-step's input is the caller's state itself: its prior-
        // mapping rewrites only the GHOST cells, whose old values never enter
        W.cur[i][0] = Buf{static_cast<float*>(const_cast<void*>(f_in[i])),
                          scalar ? const_cast<float*>(g_in[i]) : nullptr};
        bool staged = false;
        rc = prior_stage(sc, P, A[p], B[p], gA[p], gB[p], &staged, stream);
        if (rc) return rc;
        stage_used[i] = staged;
        for (int k = 1; k <= ss.last; ++k) {
            const Buf& cur = W.cur[i][k - 1];
            rc = prior_map(sc, staged, P, A[p], B[p], gA[p], gB[p], prior_weight(k, ss.l, ss.alpha),
                           cur.f, cur.g, stream);
            if (rc) return rc;
            if (k < ss.l) {
                const Buf& out = (ss.node && k == ss.last) ? W.R[i] : W.cur[i][k];
                rc = launch_step_into(L, cur.f, out.f, cur.g, out.g, stream);
            } else {
                rc = launch_step_interp(L, cur.f, W.R[i].f, cur.g, W.R[i].g, W.cur[i][0].f,
                                        W.cur[i][0].g, ss.l0, ss.l1, ss.l2, stream);
            }
            if (rc) return rc;
        }
        rc = prior_map(sc, staged, P, A[p], B[p], gA[p], gB[p], 1.0, W.R[i].f, W.R[i].g, stream);
        if (rc) return rc;
        A[i] = W.cur[i][0].f;
        gA[i] = W.cur[i][0].g;
        B[i] = W.R[i].f;
        gB[i] = W.R[i].g;
    }

    // ---- reverse ----
    hipLaunchKernelGGL(k_fill_value<int32_t>, dim3(grid_for(W.max_cells)), dim3(256), 0, stream,
                       W.gather.map, W.max_cells, -1);
    hipLaunchKernelGGL(k_fill_value<uint8_t>, dim3(grid_for(W.max_cells)), dim3(256), 0, stream,
                       W.gather.touched, W.max_cells, (uint8_t)0);
    const GatherWs* gw = &W.gather;
    // lamA[i] receives the prior-mapping adjoints of the finer scale that has
    // scale i as its parent (the reference scale always has one) and the
    // time interpolation's l0 term; a scale with neither (the finest one at
    // integer alpha) keeps it zero, and its clearing and adding are skipped
    bool uses_lamA[CSLBM_MAX_SCALES] = {};
    uses_lamA[0] = true;
    for (int i = 1; i < ns; ++i) {
        uses_lamA[S[i].parent] = true;
        if (!sub_steps(S, i).node) uses_lamA[i] = true;
    }
    // The reference scale's lamA receives only scale 1's prior-mapping
    // adjoints, inside the source sub-box scale 1's box reaches: when no
    // stencil wraps, only that sub-box is cleared here and added at the end
    // (the reference scale is the largest: clearing and summing it whole
    // moved four full buffers)
    // (a reference scale alone: lamA is never written, the box is empty)
    const SrcBox ref_box = ns > 1 ? source_box(&S[0].level, &S[1].level) : SrcBox{0, 0, 0, 0, 0, 0};
    const bool ref_boxed = ns == 1 || source_box_holds_stencils(&S[0].level, &S[1].level);
    const int planes0 = Q + (scalar ? QS : 0);
    for (int i = 0; i < ns; ++i) {
        if (!uses_lamA[i]) continue;
        if (i == 0 && ref_boxed) {
            const int64_t nb = (int64_t)ref_box.nx * ref_box.ny * ref_box.nz;
            if (nb > 0)
                hipLaunchKernelGGL(k_box_zero, dim3(grid_for(nb)), dim3(256), 0, stream, W.lamA[0].f, planes0,
                                   S[0].level.plane, S[0].level.nx, S[0].level.ny, ref_box);
        } else {
            hipLaunchKernelGGL(k_zero, dim3(grid_for(nelem(i))), dim3(256), 0, stream, W.lamA[i].f, nelem(i));
        }
    }
    for (int i = ns - 1; i >= 1; --i) {
        const cslbm_scale& sc = S[i];
        const cslbm_level* L = &sc.level;
        const cslbm_level* P = &S[i - 1].level;
        const int p = i - 1;
        const SubSteps ss = sub_steps(S, i);
        float* lamR = lam[i];
        float* muR = scalar ? mu[i] : nullptr;
        // post-mappings into the coarser scales (forward order j = 0 .. i - 1)
        for (int j = i - 1; j >= 0; --j) {
            rc = launch_exchange_adjoint(L, W.R[i].f, W.R[i].f, W.R[i].g, W.R[i].g, 0.0, &S[j].level,
                                         lam[j], scalar ? mu[j] : nullptr, lamR, nullptr, muR,
                                         nullptr, sc.post_cells[j], sc.n_post[j], gw, stream,
                                         sc.post_tiles[j], sc.n_post_tiles[j]);
            if (rc) return rc;
        }
        // the parent's columns around the shell's x-faces as the recompute
        // staged them: still in place unless another scale's stage overlaps
        // this one's (then staged again)
        bool staged = false;
        if (stage_shared(S, ns, i)) {
            rc = prior_stage(sc, P, A[p], B[p], gA[p], gB[p], &staged, stream);
            if (rc) return rc;
        } else {
            staged = stage_used[i];
        }
        // ghost shell of the interpolated state, mapped at weight 1
        rc = launch_exchange_adjoint(P, A[p], B[p], gA[p], gB[p], 1.0, L, lamR, muR, W.lamA[p].f,
                                     lam[p], W.lamA[p].g, scalar ? mu[p] : nullptr, sc.ghost_cells,
                                     sc.n_ghost, gw, stream, sc.ghost_tiles, sc.n_ghost_tiles, &sc, staged,
                                     true);
        if (rc) return rc;
        // last sub-step: R = l0 cur_1 + l1 cur_l + l2 step(cur_l), or R = step(cur_last)
        const int64_t nf = (int64_t)Q * L->plane, ngs = (int64_t)QS * L->plane;
        Buf lc = W.t1[i];
        const Buf& in_last = W.cur[i][ss.last - 1];
        rc = launch_adjoint_into(L, in_last.f, in_last.g, lamR, muR, lc.f, lc.g, nullptr, stream);
        if (rc) return rc;
        if (!ss.node) {
            // lc = l1 lamR + l2 lc and lamA += l0 lamR, lamR read once
            hipLaunchKernelGGL(k_axpby2, dim3(grid_for(nf)), dim3(256), 0, stream, lamR, lc.f, W.lamA[i].f, nf,
                               (float)ss.l1, (float)ss.l2, (float)ss.l0, 1.0f);
            if (scalar) {
                hipLaunchKernelGGL(k_axpby2, dim3(grid_for(ngs)), dim3(256), 0, stream, muR, lc.g, W.lamA[i].g,
                                   ngs, (float)ss.l1, (float)ss.l2, (float)ss.l0, 1.0f);
            }
        }
        // lam[i] is free from here on.  lc = adjoint of the input of sub-step
        // k (after its prior-map); the step adjoints below alternate between
        // lam[i] and t2 so that the last one writes lam[i].
        const Buf out_final{lamR, muR};
        for (int k = ss.last; k >= 1; --k) {
            if (k == 1 && uses_lamA[i]) {
                // the first input is also read by the interpolation and by the
                // next finer scale's prior-maps: their adjoints are in lamA[i]
                axpby(W.lamA[i].f, lc.f, nf, 1.0f, 1.0f, stream);
                if (scalar) axpby(W.lamA[i].g, lc.g, ngs, 1.0f, 1.0f, stream);
            }
            rc = launch_exchange_adjoint(P, A[p], B[p], gA[p], gB[p], prior_weight(k, ss.l, ss.alpha), L, lc.f,
                                         lc.g, W.lamA[p].f, lam[p], W.lamA[p].g,
                                         scalar ? mu[p] : nullptr, sc.ghost_cells, sc.n_ghost, gw,
                                         stream, sc.ghost_tiles, sc.n_ghost_tiles, &sc, staged, true);
            if (rc) return rc;
            if (k == 1) break;
            const Buf out = ((k - 2) % 2 == 0) ? out_final : W.t2[i];
            const Buf& in = W.cur[i][k - 2];
            rc = launch_adjoint_into(L, in.f, in.g, lc.f, lc.g, out.f, out.g, nullptr, stream);
            if (rc) return rc;
            lc = out;
        }
        // lc = dL/d(state of scale i at t_n); only a single sub-step leaves it in t1
        if (lc.f != lamR) {
            CSLBM_HIP_TRY(hipMemcpyAsync(lamR, lc.f, nf * 4, hipMemcpyDeviceToDevice, stream));
            if (scalar) CSLBM_HIP_TRY(hipMemcpyAsync(muR, lc.g, ngs * 4, hipMemcpyDeviceToDevice, stream));
        }
    }
    {
        const cslbm_level* L = &S[0].level;
        rc = launch_adjoint_into(L, f_in[0], scalar ? g_in[0] : nullptr, lam[0],
                                 scalar ? mu[0] : nullptr, W.t1[0].f, W.t1[0].g, nullptr, stream);
        if (rc) return rc;
        const int64_t nf = (int64_t)Q * L->plane, ngs = (int64_t)QS * L->plane;
        if (ref_boxed) {
            // lam[0] = t1, plus lamA[0] over the box where it can be nonzero
            const dim3 cb = step_block(L->nx);
            const dim3 cg((L->nx + cb.x - 1) / cb.x, (L->ny + cb.y - 1) / cb.y, L->nz);
            hipLaunchKernelGGL(k_copy_add_box<Q>, cg, cb, 0, stream, W.t1[0].f, W.lamA[0].f, lam[0], L->plane,
                               L->nx, L->ny, ref_box);
            if (scalar)
                hipLaunchKernelGGL(k_copy_add_box<QS>, cg, cb, 0, stream, W.t1[0].g, W.lamA[0].g, mu[0],
                                   L->plane, L->nx, L->ny, ref_box);
        } else {
            hipLaunchKernelGGL(k_sum, dim3(grid_for(nf)), dim3(256), 0, stream, W.t1[0].f, W.lamA[0].f, lam[0], nf);
            if (scalar)
                hipLaunchKernelGGL(k_sum, dim3(grid_for(ngs)), dim3(256), 0, stream, W.t1[0].g, W.lamA[0].g,
                                   mu[0], ngs);
        }
    }
    return check_launch("cslbm_multiscale_adjoint_step");
}

}  // extern "C"
