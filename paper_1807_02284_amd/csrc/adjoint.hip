// adjoint.hip -- adjoint of the collide-stream step and the store-every-step
// forward used to recompute checkpointed segments (gfx950).
//
// One step maps f(n) to f(n+1): f(n+1)(x) = C(P f(n)(x), theta(x)), with P
// the pull f_i(x) = f~_i(x - c_i) and C the local cell update.  Its adjoint
// is lam(n) = P^T J_C^T lam(n+1): each thread recomputes its cell's forward
// update from the pulled state, applies the vector-Jacobian product of
// cm_adjoint.hpp, and writes dL/df_i(x) back to the pull source (x - c_i,
// plane i).  On a periodic lattice the pull is a permutation, so every
// (plane, cell) of lam(n) is written by exactly one thread and no atomics are
// needed.  dL/dtheta(x) is accumulated by the thread that owns cell x.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/cslbm.h"
#include "cm_adjoint.hpp"
#include "cm_collide.hpp"
#include "internal.hpp"
#include "lattice.hpp"

namespace cslbm {

struct AdjArgs {
    const void* f;        // forward state f(n) (storage type)
    const float* g;       // forward scalar state g(n) or null
    const float* theta;   // [3][plane] or null
    const float* lam1;    // dL/df(n+1) [27][plane]
    const float* mu1;     // dL/dg(n+1) [7][plane] or null
    float* lam0;          // dL/df(n)
    float* mu0;           // dL/dg(n)
    float* dtheta;        // [3][plane] accumulated, or null
    int nx, ny, nz;
    int64_t plane;
    AdjointParams ap;
};

template <typename T, bool kScalar>
__global__ void __launch_bounds__(256) k_adjoint(const AdjArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz, nxy = nx * ny;
    const int cell = x + nx * y + nxy * z;
    const int64_t P = a.plane;
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int sx[3] = {xp, x, xm};
    const int sy[3] = {yp * nx, y * nx, ym * nx};
    const int sz[3] = {zp * nxy, z * nxy, zm * nxy};
    const T* f = static_cast<const T*>(a.f);

    float h[27], lam[27];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
        h[tensor_slot(i)] = Io<T>::ld(f + i * P + src);
        lam[tensor_slot(i)] = a.lam1[i * P + cell];
    }
    float gv[QS] = {0, 0, 0, 0, 0, 0, 0}, mu[QS] = {0, 0, 0, 0, 0, 0, 0};
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const int src = sx[kSx[i] + 1] + sy[kSy[i] + 1] + sz[kSz[i] + 1];
            gv[i] = a.g[i * P + src];
            mu[i] = a.mu1[i * P + cell];
        }
    }
    float th[3] = {0.0f, 0.0f, 0.0f};
    if (a.theta) {
        th[0] = a.theta[cell];
        th[1] = a.theta[P + cell];
        th[2] = a.theta[2 * P + cell];
    }
    float hb[27], gb[QS], thb[3];
    cm_collide_adjoint<kScalar>(h, gv, th, a.ap, lam, mu, hb, gb, thb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
        __builtin_nontemporal_store(hb[tensor_slot(i)], a.lam0 + i * P + src);
    }
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const int src = sx[kSx[i] + 1] + sy[kSy[i] + 1] + sz[kSz[i] + 1];
            a.mu0[i * P + src] = gb[i];
        }
    }
    if (a.dtheta) {
        a.dtheta[cell] += thb[0];
        a.dtheta[P + cell] += thb[1];
        a.dtheta[2 * P + cell] += thb[2];
    }
}

template <typename T>
static void launch_adjoint(const AdjArgs& a, bool scalar, hipStream_t st)
{
    const dim3 block = step_block(a.nx);
    const dim3 grid((a.nx + block.x - 1) / block.x, (a.ny + block.y - 1) / block.y, a.nz);
    if (scalar)
        hipLaunchKernelGGL((k_adjoint<T, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_adjoint<T, false>), grid, block, 0, st, a);
}

}  // namespace cslbm

using namespace cslbm;

extern "C" {

int cslbm_adjoint_step(const cslbm_level* L, const float* lam_next, const float* mu_next,
                       float* lam, float* mu, float* dtheta, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    rc = validate_params(L);
    if (rc) return rc;
    if ((L->periodic & 7) != 7 || L->flags)
        return fail(CSLBM_ERR_UNSUPPORTED,
                    "the adjoint step supports fully periodic levels without cell flags");
    if (L->p.grad_mode != 0)
        return fail(CSLBM_ERR_UNSUPPORTED,
                    "the adjoint step differentiates the local gradient estimate (grad_mode 0)");
    if (!lam_next || !lam) return fail(CSLBM_ERR_ARG, "adjoint buffers are NULL");
    if (lam_next == lam) return fail(CSLBM_ERR_ARG, "lam and lam_next alias");
    const bool scalar = L->g != nullptr;
    if (scalar && (!mu_next || !mu || mu == mu_next))
        return fail(CSLBM_ERR_ARG, "a level with a scalar needs distinct mu and mu_next");
    AdjArgs a;
    a.f = L->f;
    a.g = L->g;
    a.theta = L->force;
    a.lam1 = lam_next;
    a.mu1 = scalar ? mu_next : nullptr;
    a.lam0 = lam;
    a.mu0 = scalar ? mu : nullptr;
    a.dtheta = dtheta;
    a.nx = L->nx;
    a.ny = L->ny;
    a.nz = L->nz;
    a.plane = L->plane;
    a.ap.r = make_rates(L->p);
    a.ap.beta = (float)L->p.beta;
    a.ap.s_ref = (float)L->p.s_ref;
    a.ap.inv_tau_s = scalar ? (float)(1.0 / L->p.tau_s) : 0.0f;
    if (L->storage == CSLBM_F32)
        launch_adjoint<float>(a, scalar, stream);
    else
        launch_adjoint<_Float16>(a, scalar, stream);
    return check_launch("k_adjoint");
}

int cslbm_step_store(const cslbm_level* L, int32_t n_steps, void* const* f_states,
                     float* const* g_states, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    rc = validate_params(L);
    if (rc) return rc;
    if (n_steps < 0) return fail(CSLBM_ERR_ARG, "n_steps is negative");
    if (n_steps > 0 && !f_states) return fail(CSLBM_ERR_ARG, "f_states is NULL");
    if (L->g && n_steps > 0 && !g_states) return fail(CSLBM_ERR_ARG, "g_states is NULL");
    for (int k = 0; k < n_steps; ++k) {
        if (!f_states[k] || f_states[k] == (k ? f_states[k - 1] : L->f))
            return fail(CSLBM_ERR_ARG, "f_states[%d] is NULL or aliases its input", k);
        if (L->g && (!g_states[k] || g_states[k] == (k ? g_states[k - 1] : L->g)))
            return fail(CSLBM_ERR_ARG, "g_states[%d] is NULL or aliases its input", k);
    }
    for (int k = 0; k < n_steps; ++k) {
        const void* fin = k ? f_states[k - 1] : L->f;
        const float* gin = L->g ? (k ? g_states[k - 1] : L->g) : nullptr;
        rc = launch_step_into(L, fin, f_states[k], gin, L->g ? g_states[k] : nullptr, stream);
        if (rc) return rc;
    }
    return CSLBM_OK;
}

}  // extern "C"
