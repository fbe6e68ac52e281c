// cm_adjoint.hpp -- reverse mode (vector-Jacobian product) of the cell
// update in cm_collide.hpp, for the differentiable rollout.
//
// The forward cell update maps the pulled shifted populations h (27), the
// pulled scalar populations g (7) and the body force theta (3) to the
// post-collision h~ and g~.  Given the adjoints lam = dL/dh~ and
// mu = dL/dg~, cm_collide_adjoint returns dL/dh, dL/dg and dL/dtheta.  It
// recomputes the forward stages in registers and walks them backwards:
//   scalar BGK  ->  inverse sweeps K(u)^-1  ->  per-order relaxation
//   (including the adaptive factor phi(G))  ->  closed-form deviation
//   equilibria D(rho, u)  ->  forward sweeps K(u)  ->  u = (j + F/2)/rho
//   ->  F = theta + beta (s - s_ref) z.
// Non-smooth points: the clamp min(G/g_max, 1) takes the derivative of the
// branch it is on (zero once clamped), and G = sqrt(2 S^:S^) has derivative
// zero at G = 0.
#pragma once

#include <hip/hip_runtime.h>

#include "cm_collide.hpp"
#include "lattice.hpp"

namespace cslbm {

// reverse of fwd3: (b0, b1, b2) are the adjoints of the outputs (s0, k1, k2);
// am, a0, ap are the inputs; returns their adjoints in place of b*, adds the
// u adjoint to ub
__host__ __device__ __forceinline__ void fwd3_rev(float am, float a0, float ap, float u, float& b0,
                                                  float& b1, float& b2, float& ub)
{
    const float s0 = (ap + am) + a0;   // as fwd3 forms it
    const float s1 = ap - am;
    const float s0b = b0 - u * b1 + u * u * b2;
    const float s1b = b1 - 2.0f * u * b2;
    const float s2b = b2;
    ub += -s0 * b1 + (2.0f * u * s0 - 2.0f * s1) * b2;
    b0 = s0b - s1b + s2b;   // adjoint of am
    b1 = s0b;               // adjoint of a0
    b2 = s0b + s1b + s2b;   // adjoint of ap
}

// reverse of inv3: (bm, b0, bp) are the adjoints of the outputs
// (a-, a0, a+); k0, k1, k2 the inputs; returns their adjoints in place
__host__ __device__ __forceinline__ void inv3_rev(float k0, float k1, float k2, float u, float& bm,
                                                  float& b0, float& bp, float& ub)
{
    (void)k2;
    const float s2b = 0.5f * (bm + bp) - b0;
    const float s1b = 0.5f * (bp - bm);
    ub += s1b * k0 + s2b * (2.0f * k1 + 2.0f * u * k0);
    const float k0b = b0 + s1b * u + s2b * u * u;
    const float k1b = s1b + 2.0f * u * s2b;
    bm = k0b;
    b0 = k1b;
    bp = s2b;
}

template <int STRIDE, int O1, int O2>
__host__ __device__ __forceinline__ void sweep_fwd_rev(const float (&in)[27], float (&bar)[27],
                                                       float u, float& ub)
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int t = b * O1 + c * O2;
            fwd3_rev(in[t], in[t + STRIDE], in[t + 2 * STRIDE], u, bar[t], bar[t + STRIDE],
                     bar[t + 2 * STRIDE], ub);
        }
}

template <int STRIDE, int O1, int O2>
__host__ __device__ __forceinline__ void sweep_inv_rev(const float (&in)[27], float (&bar)[27],
                                                       float u, float& ub)
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int t = b * O1 + c * O2;
            inv3_rev(in[t], in[t + STRIDE], in[t + 2 * STRIDE], u, bar[t], bar[t + STRIDE],
                     bar[t + 2 * STRIDE], ub);
        }
}

// adjoint of deviation_equilibrium: adds dD/d(dr, X, Y, Z) contracted with
// db to drb, Xb, Yb, Zb (the order-0 and order-1 entries never reach the
// relaxation and are skipped)
__host__ __device__ __forceinline__ void deviation_equilibrium_rev(const float (&db)[27], float dr,
                                                                   float X, float Y, float Z,
                                                                   float& drb, float& Xb, float& Yb,
                                                                   float& Zb)
{
    const float X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    const float third = 1.0f / 3.0f, ninth = 1.0f / 9.0f;
    const float r3m1 = 2.0f + 3.0f * dr;
    const float r16 = -5.0f - 6.0f * dr;
    float b;
    // second order, off-diagonal: -AB
    b = db[kslot(1, 1, 0)]; Xb -= b * Y; Yb -= b * X;
    b = db[kslot(1, 0, 1)]; Xb -= b * Z; Zb -= b * X;
    b = db[kslot(0, 1, 1)]; Yb -= b * Z; Zb -= b * Y;
    // second order, diagonal: dr/3 - A^2
    b = db[kslot(2, 0, 0)]; drb += b * third; Xb -= 2.0f * X * b;
    b = db[kslot(0, 2, 0)]; drb += b * third; Yb -= 2.0f * Y * b;
    b = db[kslot(0, 0, 2)]; drb += b * third; Zb -= 2.0f * Z * b;
    // third order: A (1/3 - dr B^2)
#define CSLBM_D3(m, n, p, A, Ab, B, Bb)                          \
    b = db[kslot(m, n, p)];                                      \
    Ab += b * (third - dr * B * B);                              \
    Bb -= b * 2.0f * A * dr * B;                                 \
    drb -= b * A * B * B;
    CSLBM_D3(1, 2, 0, X, Xb, Y, Yb)
    CSLBM_D3(1, 0, 2, X, Xb, Z, Zb)
    CSLBM_D3(2, 1, 0, Y, Yb, X, Xb)
    CSLBM_D3(0, 1, 2, Y, Yb, Z, Zb)
    CSLBM_D3(2, 0, 1, Z, Zb, X, Xb)
    CSLBM_D3(0, 2, 1, Z, Zb, Y, Yb)
#undef CSLBM_D3
    b = db[kslot(1, 1, 1)];
    drb -= b * X * Y * Z;
    Xb -= b * dr * Y * Z;
    Yb -= b * dr * X * Z;
    Zb -= b * dr * X * Y;
    // fourth order, two squares: dr/9 - (A^2 + B^2)/3 + (3 rho - 1) A^2 B^2
#define CSLBM_D4S(m, n, p, A, Ab, B, Bb)                         \
    b = db[kslot(m, n, p)];                                      \
    drb += b * (ninth + 3.0f * A * A * B * B);                   \
    Ab += b * (-2.0f * third * A + 2.0f * r3m1 * A * B * B);     \
    Bb += b * (-2.0f * third * B + 2.0f * r3m1 * A * A * B);
    CSLBM_D4S(2, 2, 0, X, Xb, Y, Yb)
    CSLBM_D4S(2, 0, 2, X, Xb, Z, Zb)
    CSLBM_D4S(0, 2, 2, Y, Yb, Z, Zb)
#undef CSLBM_D4S
    // fourth order, one square: B C ((3 rho - 1) A^2 - 1/3)
#define CSLBM_D4P(m, n, p, A, Ab, B, Bb, Cc, Cb)                 \
    b = db[kslot(m, n, p)];                                      \
    drb += b * 3.0f * A * A * B * Cc;                            \
    Ab += b * 2.0f * r3m1 * A * B * Cc;                          \
    Bb += b * Cc * (r3m1 * A * A - third);                       \
    Cb += b * B * (r3m1 * A * A - third);
    CSLBM_D4P(2, 1, 1, X, Xb, Y, Yb, Z, Zb)
    CSLBM_D4P(1, 2, 1, Y, Yb, X, Xb, Z, Zb)
    CSLBM_D4P(1, 1, 2, Z, Zb, X, Xb, Y, Yb)
#undef CSLBM_D4P
    // fifth order: A (1/9 - dr (B^2 + C^2)/3 + (1 - 6 rho) B^2 C^2)
#define CSLBM_D5(m, n, p, A, Ab, B, Bb, Cc, Cb)                                        \
    b = db[kslot(m, n, p)];                                                            \
    drb += b * A * (-(B * B + Cc * Cc) * third - 6.0f * B * B * Cc * Cc);              \
    Ab += b * (ninth - dr * (B * B + Cc * Cc) * third + r16 * B * B * Cc * Cc);        \
    Bb += b * A * (-2.0f * dr * B * third + 2.0f * r16 * B * Cc * Cc);                 \
    Cb += b * A * (-2.0f * dr * Cc * third + 2.0f * r16 * B * B * Cc);
    CSLBM_D5(1, 2, 2, X, Xb, Y, Yb, Z, Zb)
    CSLBM_D5(2, 1, 2, Y, Yb, X, Xb, Z, Zb)
    CSLBM_D5(2, 2, 1, Z, Zb, X, Xb, Y, Yb)
#undef CSLBM_D5
    // sixth order
    b = db[kslot(2, 2, 2)];
    {
        const float q = X2 * Y2 + X2 * Z2 + Y2 * Z2;
        const float c2 = 2.0f * third + dr;
        const float c3 = 9.0f + 10.0f * dr;
        drb += b * (1.0f / 27.0f + q + 10.0f * X2 * Y2 * Z2);
        Xb += b * (-2.0f * ninth * X + c2 * 2.0f * X * (Y2 + Z2) + c3 * 2.0f * X * Y2 * Z2);
        Yb += b * (-2.0f * ninth * Y + c2 * 2.0f * Y * (X2 + Z2) + c3 * 2.0f * Y * X2 * Z2);
        Zb += b * (-2.0f * ninth * Z + c2 * 2.0f * Z * (X2 + Y2) + c3 * 2.0f * Z * X2 * Y2);
    }
}

struct AdjointParams {
    Rates r;
    float beta, s_ref, inv_tau_s;
};

// Vector-Jacobian product of one cell update.
//   h[27]   pulled shifted populations (tensor order), gv[7] pulled scalar
//           populations (ignored unless kScalar), th[3] body force theta
//   lam[27] dL/dh~ (tensor order), mu[7] dL/dg~
// Outputs: hb[27] = dL/dh (tensor order), gb[7] = dL/dg, thb[3] = dL/dtheta.
template <bool kScalar>
__host__ __device__ __forceinline__ void cm_collide_adjoint(const float (&h)[27], const float (&gv)[7],
                                                            const float (&th)[3],
                                                            const AdjointParams& ap,
                                                            const float (&lam)[27],
                                                            const float (&mu)[7], float (&hb)[27],
                                                            float (&gb)[7], float (&thb)[3])
{
    const Rates& r = ap.r;
    // ---------------- forward recomputation ----------------
    float s = 0.0f;
    if (kScalar) s = (gv[0] + (gv[1] + gv[2])) + ((gv[3] + gv[4]) + (gv[5] + gv[6]));
    const float Fx = th[0], Fy = th[1];
    const float Fz = th[2] + (kScalar ? ap.beta * (s - ap.s_ref) : 0.0f);
    float dr, jx, jy, jz;
    moments0(h, dr, jx, jy, jz);
    const float rho = 1.0f + dr;
    const float ir = 1.0f / rho;
    const float ux = (jx + 0.5f * Fx) * ir;
    const float uy = (jy + 0.5f * Fy) * ir;
    const float uz = (jz + 0.5f * Fz) * ir;

    // group of every moment of order >= 3 (-1: orders 0..2, handled apart)
    constexpr int kGroup[27] = {
        // m + 3n + 9p -> group by total order (3 -> 0, 4 -> 1, 5 -> 2, 6 -> 3)
        -1, -1, -1, -1, -1, 0, -1, 0, 1,     // p = 0: 000 100 200 010 110 210 020 120 220
        -1, -1, 0, -1, 0, 1, 0, 1, 2,        // p = 1: 001 101 201 011 111 211 021 121 221
        -1, 0, 1, 0, 1, 2, 1, 2, 3};         // p = 2: 002 102 202 012 112 212 022 122 222

    // forward moments v = K(u) h, deviation equilibria d, adaptive rates and
    // the post-collision moments w; v and d are recomputed later instead of
    // being kept live through the reverse sweeps (register pressure)
    float w[27];
    float nxy, nxz, nyz, tr, pxx, pyy, pzz, pp, sq, G, phi = 1.0f;
    bool on_slope = false;
    float om[4], den[4];
    const float oms = 1.0f - r.S;
    {
        float d[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) w[q] = h[q];
        to_moments(w, ux, uy, uz);
        deviation_equilibrium(d, dr, ux, uy, uz);
        nxy = w[kslot(1, 1, 0)] - d[kslot(1, 1, 0)];
        nxz = w[kslot(1, 0, 1)] - d[kslot(1, 0, 1)];
        nyz = w[kslot(0, 1, 1)] - d[kslot(0, 1, 1)];
        const float nxx = w[kslot(2, 0, 0)] - d[kslot(2, 0, 0)];
        const float nyy = w[kslot(0, 2, 0)] - d[kslot(0, 2, 0)];
        const float nzz = w[kslot(0, 0, 2)] - d[kslot(0, 0, 2)];
        tr = (nxx + nyy + nzz) * (1.0f / 3.0f);
        pxx = nxx - tr;
        pyy = nyy - tr;
        pzz = nzz - tr;
        pp = pxx * pxx + pyy * pyy + pzz * pzz + 2.0f * (nxy * nxy + nxz * nxz + nyz * nyz);
        sq = sqrtf(2.0f * pp);
        G = 1.5f * r.S * ir * sq;
        if (r.adaptive) {
            const float xg = G * r.inv_gmax;
            on_slope = xg < 1.0f;
            phi = r.a * fminf(xg, 1.0f) + r.b;
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            den[g] = phi * r.nu3[g] + 0.5f;
            om[g] = 1.0f - 1.0f / den[g];
        }
        w[kslot(1, 0, 0)] += Fx;
        w[kslot(0, 1, 0)] += Fy;
        w[kslot(0, 0, 1)] += Fz;
        w[kslot(1, 1, 0)] = d[kslot(1, 1, 0)] + oms * nxy;
        w[kslot(1, 0, 1)] = d[kslot(1, 0, 1)] + oms * nxz;
        w[kslot(0, 1, 1)] = d[kslot(0, 1, 1)] + oms * nyz;
        w[kslot(2, 0, 0)] = d[kslot(2, 0, 0)] + oms * pxx + om[0] * tr;
        w[kslot(0, 2, 0)] = d[kslot(0, 2, 0)] + oms * pyy + om[0] * tr;
        w[kslot(0, 0, 2)] = d[kslot(0, 0, 2)] + oms * pzz + om[0] * tr;
#pragma unroll
        for (int q = 0; q < 27; ++q)
            if (kGroup[q] >= 0) w[q] = d[q] + om[kGroup[q]] * (w[q] - d[q]);
    }

    // ---------------- reverse ----------------
    float uxb = 0.0f, uyb = 0.0f, uzb = 0.0f, sb = 0.0f;

    // scalar BGK: g~ = (1 - 1/tau) g + (1/tau) g^eq(s, u)
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            gb[i] = (1.0f - ap.inv_tau_s) * mu[i];
            const float me = ap.inv_tau_s * mu[i];
            const float cu = kSx[i] * ux + kSy[i] * uy + kSz[i] * uz;
            sb += me * kSw[i] * (1.0f + 4.0f * cu);
            const float su = me * kSw[i] * s * 4.0f;
            uxb += su * kSx[i];
            uyb += su * kSy[i];
            uzb += su * kSz[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < QS; ++i) gb[i] = 0.0f;
    }

    // inverse sweeps: h~ = Ix(Iy(Iz(w))); the sweep inputs are rebuilt from w
    // one at a time rather than kept together (register pressure)
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
    // bar = dL/dw

    // relaxation (v and d recomputed)
    float vb[27], db[27];
    float omb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    {
        float v[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) v[q] = h[q];
        to_moments(v, ux, uy, uz);
        deviation_equilibrium(db, dr, ux, uy, uz);   // db holds d for a moment
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            if (kGroup[q] >= 0) {
                const int g = kGroup[q];
                omb[g] += (v[q] - db[q]) * bar[q];
                vb[q] = om[g] * bar[q];
                db[q] = (1.0f - om[g]) * bar[q];
            } else {
                vb[q] = 0.0f;
                db[q] = 0.0f;
            }
        }
    }
    vb[kslot(0, 0, 0)] = bar[kslot(0, 0, 0)];
    vb[kslot(1, 0, 0)] = bar[kslot(1, 0, 0)];
    vb[kslot(0, 1, 0)] = bar[kslot(0, 1, 0)];
    vb[kslot(0, 0, 1)] = bar[kslot(0, 0, 1)];
    float Fxb = bar[kslot(1, 0, 0)], Fyb = bar[kslot(0, 1, 0)], Fzb = bar[kslot(0, 0, 1)];
    float phib = 0.0f;
    // second order: off-diagonal and diagonal (deviatoric with S, trace with om0)
    float nxyb = oms * bar[kslot(1, 1, 0)], nxzb = oms * bar[kslot(1, 0, 1)],
          nyzb = oms * bar[kslot(0, 1, 1)];
    db[kslot(1, 1, 0)] += bar[kslot(1, 1, 0)];
    db[kslot(1, 0, 1)] += bar[kslot(1, 0, 1)];
    db[kslot(0, 1, 1)] += bar[kslot(0, 1, 1)];
    const float bxx = bar[kslot(2, 0, 0)], byy = bar[kslot(0, 2, 0)], bzz = bar[kslot(0, 0, 2)];
    db[kslot(2, 0, 0)] += bxx;
    db[kslot(0, 2, 0)] += byy;
    db[kslot(0, 0, 2)] += bzz;
    const float bsum = bxx + byy + bzz;
    omb[0] += tr * bsum;
    // w_a = oms (n_a - tr) + om0 tr  ->  n_a adjoint
    float nxxb = oms * bxx + (om[0] - oms) * bsum * (1.0f / 3.0f);
    float nyyb = oms * byy + (om[0] - oms) * bsum * (1.0f / 3.0f);
    float nzzb = oms * bzz + (om[0] - oms) * bsum * (1.0f / 3.0f);
    // adaptive factor: om_g = 1 - 1/(phi nu3_g + 1/2)
#pragma unroll
    for (int g = 0; g < 4; ++g) phib += omb[g] * r.nu3[g] / (den[g] * den[g]);
    if (r.adaptive && on_slope && pp > 0.0f) {
        const float Gb = phib * r.a * r.inv_gmax;
        // G = 1.5 S ir sqrt(2 pp)
        const float ppb = Gb * 1.5f * r.S * ir / sq;
        const float irb_g = Gb * 1.5f * r.S * sq;
        // pp = sum p_a^2 + 2 (nxy^2 + nxz^2 + nyz^2), p_a = n_a - tr
        const float pxxb = 2.0f * pxx * ppb, pyyb = 2.0f * pyy * ppb, pzzb = 2.0f * pzz * ppb;
        const float pm = (pxxb + pyyb + pzzb) * (1.0f / 3.0f);
        nxxb += pxxb - pm;
        nyyb += pyyb - pm;
        nzzb += pzzb - pm;
        nxyb += 4.0f * nxy * ppb;
        nxzb += 4.0f * nxz * ppb;
        nyzb += 4.0f * nyz * ppb;
        // G also depends on rho through ir: d(ir)/d(dr) = -ir^2.  The D000
        // slot of db is never used by the relaxation, so it carries this
        // dr adjoint to the equilibrium stage below.
        db[kslot(0, 0, 0)] += -irb_g * ir * ir;
    }
    // n = v - d
    vb[kslot(1, 1, 0)] += nxyb;
    vb[kslot(1, 0, 1)] += nxzb;
    vb[kslot(0, 1, 1)] += nyzb;
    vb[kslot(2, 0, 0)] += nxxb;
    vb[kslot(0, 2, 0)] += nyyb;
    vb[kslot(0, 0, 2)] += nzzb;
    db[kslot(1, 1, 0)] -= nxyb;
    db[kslot(1, 0, 1)] -= nxzb;
    db[kslot(0, 1, 1)] -= nyzb;
    db[kslot(2, 0, 0)] -= nxxb;
    db[kslot(0, 2, 0)] -= nyyb;
    db[kslot(0, 0, 2)] -= nzzb;

    // deviation equilibria D(dr, u) (the D000 slot holds the dr adjoint of G)
    float drb = db[kslot(0, 0, 0)];
    deviation_equilibrium_rev(db, dr, ux, uy, uz, drb, uxb, uyb, uzb);

    // forward sweeps: v = Fz(Fy(Fx(h))), inputs rebuilt from h one at a time
    {
        float t[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) t[q] = h[q];
        sweep_fwd<1, 3, 9>(t, ux);
        sweep_fwd<3, 1, 9>(t, uy);
        sweep_fwd_rev<9, 1, 3>(t, vb, uz, uzb);
#pragma unroll
        for (int q = 0; q < 27; ++q) t[q] = h[q];
        sweep_fwd<1, 3, 9>(t, ux);
        sweep_fwd_rev<3, 1, 9>(t, vb, uy, uyb);
        sweep_fwd_rev<1, 3, 9>(h, vb, ux, uxb);
    }
    // vb = dL/dh through the transforms

    // u = (j + F/2) ir
    const float jxb = uxb * ir, jyb = uyb * ir, jzb = uzb * ir;
    Fxb += 0.5f * jxb;
    Fyb += 0.5f * jyb;
    Fzb += 0.5f * jzb;
    const float irb = uxb * (jx + 0.5f * Fx) + uyb * (jy + 0.5f * Fy) + uzb * (jz + 0.5f * Fz);
    drb += -irb * ir * ir;
    // dr = sum h, j = sum c h
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int cx = t % 3 - 1, cy = (t / 3) % 3 - 1, cz = t / 9 - 1;
        hb[t] = vb[t] + drb + cx * jxb + cy * jyb + cz * jzb;
    }
    // F = theta + beta (s - s_ref) z,  s = sum g
    thb[0] = Fxb;
    thb[1] = Fyb;
    thb[2] = Fzb;
    if (kScalar) {
        sb += ap.beta * Fzb;
#pragma unroll
        for (int i = 0; i < QS; ++i) gb[i] += sb;
    }
}

}  // namespace cslbm
