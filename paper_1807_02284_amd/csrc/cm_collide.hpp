// cm_collide.hpp -- register-resident central-moment collision for gfx950.
//
// The cell's 27 values are the shifted populations h_i = f_i - w_i in tensor
// order (lattice.hpp).  The collision of the paper (eq. cmr_collision,
// Omega = -T S (m - m^eq), appendix rates) is evaluated without forming the
// 27x27 matrices:
//
//   * m = M^T f is a fixed +-1 recombination B of the raw central moments
//     k_mnp = sum_i f_i (c_ix-u_x)^m (c_iy-u_y)^n (c_iz-u_z)^p.  The
//     recombination only mixes moments of one total order, and every order
//     group shares one rate, except the second-order diagonal triple where
//     m7, m8 (deviatoric part) relax with S and m9 (trace) with the m9 rate.
//     Relaxing m with S is therefore relaxing k per order, and
//     T = (M^T)^{-1} = K(u)^{-1} B^{-1} needs no inverse of B at all.
//   * k = K(u) f factorises into 3-point sweeps along x, y and z; K(u)^{-1}
//     likewise.
//   * All arithmetic is on deviations: dk = K(u) h, and the equilibrium
//     enters as D = k^eq - K(u) w, written out in closed form so that no
//     O(1) quantity is ever subtracted from another.  FP32 rounding then
//     scales with |h|, not with |f|.
//
// Equilibrium central moments: the appendix list, which equals K(u) applied
// to the second-order polynomial equilibrium; in k form:
//   k000 = rho, k200 = rho/3, k120 = -rho ux uy^2, k111 = -rho ux uy uz,
//   k220 = 3 rho ux^2 uy^2 + rho/9, k211 = 3 rho ux^2 uy uz,
//   k122 = -(rho/3) ux (18 uy^2 uz^2 + uy^2 + uz^2),
//   k222 = rho (10 ux^2 uy^2 uz^2 + ux^2 uy^2 + ux^2 uz^2 + uy^2 uz^2 + 1/27)
// and permutations; the remaining ones vanish.  K(u) w factorises into the
// 1D moments (1, -u, 1/3 + u^2) of the weights (1/6, 2/3, 1/6).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace cslbm {

// Per-level relaxation constants, precomputed on the host.
struct Rates {
    float S;          // S4..S8 = 1/(3 nu + 1/2)
    float nu3[4];     // 3 nu'_g for the groups m9..16, m17..22, m23..25, m26
    float a, b;       // adaptive model parameters
    float inv_gmax;   // 1 / g_max
    int adaptive;     // 0: phi = 1
};

// forward 3-point sweep: populations at c = -1, 0, +1 -> central moments of
// order 0, 1, 2 about u
__host__ __device__ __forceinline__ void fwd3(float& am, float& a0, float& ap, float u)
{
    const float s2 = ap + am;
    const float s0 = s2 + a0;
    const float s1 = ap - am;
    const float k1 = s1 - u * s0;
    const float k2 = s2 - u * (s1 + k1);
    am = s0;
    a0 = k1;
    ap = k2;
}

// inverse 3-point sweep: central moments of order 0, 1, 2 about u ->
// populations at c = -1, 0, +1
__host__ __device__ __forceinline__ void inv3(float& x0, float& x1, float& x2, float u)
{
    const float k0 = x0, k1 = x1, k2 = x2;
    const float s1 = k1 + u * k0;
    const float s2 = k2 + u * (k1 + s1);
    x0 = 0.5f * (s2 - s1);
    x1 = k0 - s2;
    x2 = 0.5f * (s2 + s1);
}

// inv3 with its outputs doubled: the factors 0.5 drop out.  Scaling by a
// power of two is exact, so a chain of these followed by inv3_quarter gives
// inv3's results bit for bit.
__host__ __device__ __forceinline__ void inv3_double(float& x0, float& x1, float& x2, float u)
{
    const float k0 = x0, k1 = x1, k2 = x2;
    const float s1 = k1 + u * k0;
    const float s2 = k2 + u * (k1 + s1);
    const float d = k0 - s2;
    x0 = s2 - s1;
    x1 = d + d;
    x2 = s2 + s1;
}

// inv3 of inputs scaled by 4 (after two doubled sweeps), outputs unscaled
__host__ __device__ __forceinline__ void inv3_quarter(float& x0, float& x1, float& x2, float u)
{
    const float k0 = x0, k1 = x1, k2 = x2;
    const float s1 = k1 + u * k0;
    const float s2 = k2 + u * (k1 + s1);
    x0 = 0.125f * (s2 - s1);
    x1 = 0.25f * (k0 - s2);
    x2 = 0.125f * (s2 + s1);
}

template <int STRIDE, int O1, int O2>
__host__ __device__ __forceinline__ void sweep_fwd(float (&v)[27], float u)
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int t = b * O1 + c * O2;
            fwd3(v[t], v[t + STRIDE], v[t + 2 * STRIDE], u);
        }
}

template <int STRIDE, int O1, int O2>
__host__ __device__ __forceinline__ void sweep_inv(float (&v)[27], float u)
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int t = b * O1 + c * O2;
            inv3(v[t], v[t + STRIDE], v[t + 2 * STRIDE], u);
        }
}

__host__ __device__ __forceinline__ void to_moments(float (&v)[27], float ux, float uy, float uz)
{
    sweep_fwd<1, 3, 9>(v, ux);
    sweep_fwd<3, 1, 9>(v, uy);
    sweep_fwd<9, 1, 3>(v, uz);
}

// The x sweep split in two.  Its first half does not depend on u: every
// x-line (a-, a0, a+) becomes (s0, s1, s2) = (a- + a0 + a+, a+ - a-, a+ + a-).
// The macroscopic moments are sums of these line values, so the collision
// forms them there instead of summing the 27 populations three times over.
// (Written as fma(a, one, b) with a run-time one, these sums take binary16
// operands straight into v_fma_mix_f32 without converts: 27 fewer VALU
// instructions, but measured 3 % slower.)
__host__ __device__ __forceinline__ void xsweep_sums(float (&v)[27])
{
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        const int t = 3 * l;
        const float am = v[t], a0 = v[t + 1], ap = v[t + 2];
        const float s2 = ap + am;
        v[t] = s2 + a0;
        v[t + 1] = ap - am;
        v[t + 2] = s2;
    }
}

// dr = sum h, j = sum c h from the line values of xsweep_sums (line l = 3
// (cz + 1) + (cy + 1) starts at slot 3 l)
__host__ __device__ __forceinline__ void moments_of_sums(const float (&v)[27], float& dr, float& jx,
                                                         float& jy, float& jz)
{
    float s[9], d[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        s[l] = v[3 * l];
        d[l] = v[3 * l + 1];
    }
    dr = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])) + s[8];
    jx = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    jy = ((s[2] - s[0]) + (s[5] - s[3])) + (s[8] - s[6]);
    jz = ((s[6] - s[0]) + (s[7] - s[1])) + (s[8] - s[2]);
}

// second half of the x sweep: (s0, s1, s2) -> central moments (k0, k1, k2)
// about u, as fwd3 finishes them
__host__ __device__ __forceinline__ void xsweep_finish(float (&v)[27], float u)
{
#pragma unroll
    for (int l = 0; l < 9; ++l) {
        const int t = 3 * l;
        const float s0 = v[t], s1 = v[t + 1], s2 = v[t + 2];
        const float k1 = s1 - u * s0;
        v[t + 1] = k1;
        v[t + 2] = s2 - u * (s1 + k1);
    }
}

// inverse sweeps z and y doubled, x with the quarter: equal to sweep_inv
// along z, y, x bit for bit, with 18 fewer multiplications
template <int STRIDE, int O1, int O2, bool kLast>
__host__ __device__ __forceinline__ void sweep_inv_scaled(float (&v)[27], float u)
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int t = b * O1 + c * O2;
            if (kLast)
                inv3_quarter(v[t], v[t + STRIDE], v[t + 2 * STRIDE], u);
            else
                inv3_double(v[t], v[t + STRIDE], v[t + 2 * STRIDE], u);
        }
}

__host__ __device__ __forceinline__ void from_moments(float (&v)[27], float ux, float uy, float uz)
{
    sweep_inv_scaled<9, 1, 3, false>(v, uz);
    sweep_inv_scaled<3, 1, 9, false>(v, uy);
    sweep_inv_scaled<1, 3, 9, true>(v, ux);
}

// D = k^eq(rho, u) - K(u) w for every moment, dr = rho - 1.  Order-1 entries
// are u (k^eq vanishes, K(u) w gives -u).
__host__ __device__ __forceinline__ void deviation_equilibrium(float (&d)[27], float dr, float X, float Y,
                                                      float Z)
{
    const float X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    const float third = 1.0f / 3.0f, ninth = 1.0f / 9.0f;
    const float r3m1 = 2.0f + 3.0f * dr;   // 3 rho - 1
    const float r16 = -5.0f - 6.0f * dr;   // 1 - 6 rho
    d[kslot(0, 0, 0)] = dr;
    d[kslot(1, 0, 0)] = X;
    d[kslot(0, 1, 0)] = Y;
    d[kslot(0, 0, 1)] = Z;
    d[kslot(1, 1, 0)] = -X * Y;
    d[kslot(1, 0, 1)] = -X * Z;
    d[kslot(0, 1, 1)] = -Y * Z;
    d[kslot(2, 0, 0)] = dr * third - X2;
    d[kslot(0, 2, 0)] = dr * third - Y2;
    d[kslot(0, 0, 2)] = dr * third - Z2;
    d[kslot(1, 2, 0)] = X * (third - dr * Y2);
    d[kslot(1, 0, 2)] = X * (third - dr * Z2);
    d[kslot(2, 1, 0)] = Y * (third - dr * X2);
    d[kslot(0, 1, 2)] = Y * (third - dr * Z2);
    d[kslot(2, 0, 1)] = Z * (third - dr * X2);
    d[kslot(0, 2, 1)] = Z * (third - dr * Y2);
    d[kslot(1, 1, 1)] = -dr * X * Y * Z;
    d[kslot(2, 2, 0)] = dr * ninth - (X2 + Y2) * third + r3m1 * X2 * Y2;
    d[kslot(2, 0, 2)] = dr * ninth - (X2 + Z2) * third + r3m1 * X2 * Z2;
    d[kslot(0, 2, 2)] = dr * ninth - (Y2 + Z2) * third + r3m1 * Y2 * Z2;
    d[kslot(2, 1, 1)] = Y * Z * (r3m1 * X2 - third);
    d[kslot(1, 2, 1)] = X * Z * (r3m1 * Y2 - third);
    d[kslot(1, 1, 2)] = X * Y * (r3m1 * Z2 - third);
    d[kslot(1, 2, 2)] = X * (ninth - dr * (Y2 + Z2) * third + r16 * Y2 * Z2);
    d[kslot(2, 1, 2)] = Y * (ninth - dr * (X2 + Z2) * third + r16 * X2 * Z2);
    d[kslot(2, 2, 1)] = Z * (ninth - dr * (X2 + Y2) * third + r16 * X2 * Y2);
    d[kslot(2, 2, 2)] = dr * (1.0f / 27.0f) - (X2 + Y2 + Z2) * ninth +
                        (2.0f * third + dr) * (X2 * Y2 + X2 * Z2 + Y2 * Z2) +
                        (9.0f + 10.0f * dr) * X2 * Y2 * Z2;
}

// Macroscopic moments of shifted populations in tensor order:
// dr = sum h, j = sum c h.
__host__ __device__ __forceinline__ void moments0(const float (&v)[27], float& dr, float& jx, float& jy,
                                         float& jz)
{
    float sx[3] = {0.f, 0.f, 0.f}, sy[3] = {0.f, 0.f, 0.f}, sz[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        sx[t % 3] += v[t];
        sy[(t / 3) % 3] += v[t];
        sz[t / 9] += v[t];
    }
    dr = (sx[0] + sx[2]) + sx[1];
    jx = sx[2] - sx[0];
    jy = sy[2] - sy[0];
    jz = sz[2] - sz[0];
}

// Reciprocal: the hardware v_rcp_f32 on the device (about 1 ulp; measured
// faster than the correctly rounded division in the binary16 kernel, same
// in the FP32 one), the plain division on the host.
__host__ __device__ __forceinline__ float rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

struct CellMacro {
    float rho, ux, uy, uz, G, phi;
};

// Central-moment collision of one cell, in place on shifted populations.
// F is the body force (zero when absent): u = (j + F/2)/rho and the
// order-one central moments receive +F (source (I - S/2) R with S_1..3 = 0).
// active == false relaxes nothing (the transform pair is then an identity up
// to rounding); kernels use it for lanes of non-fluid cells.  g_given >= 0
// replaces the cell's own estimate of the gradient magnitude G.
__host__ __device__ __forceinline__ CellMacro cm_collide(float (&v)[27], const Rates& r, float Fx, float Fy,
                                               float Fz, bool active = true, float g_given = -1.0f)
{
    float dr, jx, jy, jz;
    xsweep_sums(v);
    moments_of_sums(v, dr, jx, jy, jz);
    const float rho = 1.0f + dr;
    const float inv_rho = rcp(rho);
    const float ux = (jx + 0.5f * Fx) * inv_rho;
    const float uy = (jy + 0.5f * Fy) * inv_rho;
    const float uz = (jz + 0.5f * Fz) * inv_rho;

    xsweep_finish(v, ux);
    sweep_fwd<3, 1, 9>(v, uy);
    sweep_fwd<9, 1, 3>(v, uz);
    float d[27];
    deviation_equilibrium(d, dr, ux, uy, uz);

    // non-equilibrium part n = dk - D of the second-order moments
    const float nxy = v[kslot(1, 1, 0)] - d[kslot(1, 1, 0)];
    const float nxz = v[kslot(1, 0, 1)] - d[kslot(1, 0, 1)];
    const float nyz = v[kslot(0, 1, 1)] - d[kslot(0, 1, 1)];
    const float nxx = v[kslot(2, 0, 0)] - d[kslot(2, 0, 0)];
    const float nyy = v[kslot(0, 2, 0)] - d[kslot(0, 2, 0)];
    const float nzz = v[kslot(0, 0, 2)] - d[kslot(0, 0, 2)];
    const float tr = (nxx + nyy + nzz) * (1.0f / 3.0f);
    const float pxx = nxx - tr, pyy = nyy - tr, pzz = nzz - tr;

    // adaptive relaxation: G = sqrt(2 S^:S^), S^ = -(3 S / (2 rho)) Pi_dev
    const float pp = pxx * pxx + pyy * pyy + pzz * pzz + 2.0f * (nxy * nxy + nxz * nxz + nyz * nyz);
    const float G = g_given >= 0.0f ? g_given : 1.5f * r.S * inv_rho * sqrtf(2.0f * pp);
    float phi = 1.0f;
    if (r.adaptive) phi = r.a * fminf(G * r.inv_gmax, 1.0f) + r.b;
    float om[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) om[g] = active ? 1.0f - rcp(phi * r.nu3[g] + 0.5f) : 1.0f;
    const float om_s = active ? 1.0f - r.S : 1.0f;

    // relax: dk* = D + (1 - S)(dk - D); conserved moments unchanged, +F
    v[kslot(1, 0, 0)] += Fx;
    v[kslot(0, 1, 0)] += Fy;
    v[kslot(0, 0, 1)] += Fz;
    v[kslot(1, 1, 0)] = d[kslot(1, 1, 0)] + om_s * nxy;
    v[kslot(1, 0, 1)] = d[kslot(1, 0, 1)] + om_s * nxz;
    v[kslot(0, 1, 1)] = d[kslot(0, 1, 1)] + om_s * nyz;
    const float trr = om[0] * tr;
    v[kslot(2, 0, 0)] = d[kslot(2, 0, 0)] + om_s * pxx + trr;
    v[kslot(0, 2, 0)] = d[kslot(0, 2, 0)] + om_s * pyy + trr;
    v[kslot(0, 0, 2)] = d[kslot(0, 0, 2)] + om_s * pzz + trr;
#define CSLBM_RELAX(m, n, p, g) \
    v[kslot(m, n, p)] = d[kslot(m, n, p)] + om[g] * (v[kslot(m, n, p)] - d[kslot(m, n, p)])
    CSLBM_RELAX(1, 2, 0, 0);
    CSLBM_RELAX(1, 0, 2, 0);
    CSLBM_RELAX(2, 1, 0, 0);
    CSLBM_RELAX(0, 1, 2, 0);
    CSLBM_RELAX(2, 0, 1, 0);
    CSLBM_RELAX(0, 2, 1, 0);
    CSLBM_RELAX(1, 1, 1, 0);
    CSLBM_RELAX(2, 2, 0, 1);
    CSLBM_RELAX(2, 0, 2, 1);
    CSLBM_RELAX(0, 2, 2, 1);
    CSLBM_RELAX(2, 1, 1, 1);
    CSLBM_RELAX(1, 2, 1, 1);
    CSLBM_RELAX(1, 1, 2, 1);
    CSLBM_RELAX(1, 2, 2, 2);
    CSLBM_RELAX(2, 1, 2, 2);
    CSLBM_RELAX(2, 2, 1, 2);
    CSLBM_RELAX(2, 2, 2, 3);
#undef CSLBM_RELAX

    from_moments(v, ux, uy, uz);
    return CellMacro{rho, ux, uy, uz, G, phi};
}

// Shifted equilibrium populations h^eq = T m^eq(rho, u) - w (initialisation
// section: f_0 = T m^eq), in tensor order.
__host__ __device__ __forceinline__ void shifted_equilibrium(float (&v)[27], float rho, float ux, float uy,
                                                    float uz)
{
    deviation_equilibrium(v, rho - 1.0f, ux, uy, uz);
    from_moments(v, ux, uy, uz);
}

}  // namespace cslbm
