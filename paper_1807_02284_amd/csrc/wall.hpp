// wall.hpp -- the no-slip wall node (kind kWall) of the collide-stream step.
//
// Section "Initialization and boundary treatment" uses the second-order
// no-slip wall of Latt et al. instead of bounce-back.  It is written here as
// the regularized boundary condition of Latt & Chopard (Math. Comput. Simul.
// 72, 2006) and Latt, Chopard, Malaspinas, Deville & Michler ("Straight
// velocity boundaries in the lattice Boltzmann method", Phys. Rev. E 77,
// 056703, 2008) for a flat wall that passes through the node:
//   rho   from mass and normal momentum: the populations moving along the
//         wall count once, those moving into it twice (the ones coming out
//         of it are unknown);
//   f^neq of an unknown population = f^neq of the opposite one;
//   Pi    = sum_i c_i c_i f^neq_i, and every population is rebuilt as
//         f^eq(rho, u_w) + w_i / (2 cs^4) (c_i c_i - cs^2 I) : Pi.
// With the half-force velocity shift of the collision the node's velocity
// (j + F/2)/rho is zero when its momentum is -F/2, so u_w = -F/(2 rho).
#pragma once

#include "lattice.hpp"

namespace cslbm {

// v: shifted populations h = f - w of one node in tensor order; code 1..6:
// wall normal (from the node into the wall) -x, +x, -y, +y, -z, +z.
__device__ __forceinline__ void wall_regularize(float (&v)[27], int code, float Fx, float Fy,
                                                float Fz)
{
    const int axis = (code - 1) >> 1;
    const int sgn = (code & 1) ? -1 : 1;
    const float Fn = (float)sgn * (axis == 0 ? Fx : (axis == 1 ? Fy : Fz));
    // rho - 1 (the weights of the counted populations sum to 2/3 + 2/6 = 1)
    float drho = 0.5f * Fn;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int c[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
        const int cn = sgn * (axis == 0 ? c[0] : (axis == 1 ? c[1] : c[2]));
        drho += (cn == 0 ? 1.0f : (cn > 0 ? 2.0f : 0.0f)) * v[t];
    }
    const float rho = 1.0f + drho;
    const float k = -0.5f / rho;
    const float ux = k * Fx, uy = k * Fy, uz = k * Fz;
    const float uu = ux * ux + uy * uy + uz * uz;
    // stress of the non-equilibrium part: known populations along the wall
    // once, those moving into it twice (they stand in for their opposites)
    float pxx = 0.0f, pyy = 0.0f, pzz = 0.0f, pxy = 0.0f, pxz = 0.0f, pyz = 0.0f;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int c[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
        const int cn = sgn * (axis == 0 ? c[0] : (axis == 1 ? c[1] : c[2]));
        const float w = weight1d(c[0]) * weight1d(c[1]) * weight1d(c[2]);
        const float cu = c[0] * ux + c[1] * uy + c[2] * uz;
        const float heq = w * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
        const float nq = (cn == 0 ? 1.0f : (cn > 0 ? 2.0f : 0.0f)) * (v[t] - heq);
        pxx += (float)(c[0] * c[0]) * nq;
        pyy += (float)(c[1] * c[1]) * nq;
        pzz += (float)(c[2] * c[2]) * nq;
        pxy += (float)(c[0] * c[1]) * nq;
        pxz += (float)(c[0] * c[2]) * nq;
        pyz += (float)(c[1] * c[2]) * nq;
    }
    const float tr3 = (pxx + pyy + pzz) * (1.0f / 3.0f);
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int c[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
        const float w = weight1d(c[0]) * weight1d(c[1]) * weight1d(c[2]);
        const float cu = c[0] * ux + c[1] * uy + c[2] * uz;
        const float heq = w * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
        const float qp = (float)(c[0] * c[0]) * pxx + (float)(c[1] * c[1]) * pyy +
                         (float)(c[2] * c[2]) * pzz +
                         2.0f * ((float)(c[0] * c[1]) * pxy + (float)(c[0] * c[2]) * pxz +
                                 (float)(c[1] * c[2]) * pyz) -
                         tr3;
        v[t] = heq + 4.5f * w * qp;
    }
}

}  // namespace cslbm
