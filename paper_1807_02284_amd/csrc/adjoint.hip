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
//
// Levels with cell kinds: a fluid cell pulls (x - c_i, i), or its own
// opposite population (x, opp(i)) across a bounce-back link; no two fluid
// cells pull the same element, so the fluid pass still writes without
// atomics.  Elements no fluid cell pulls have adjoint zero, written by the
// passes themselves instead of clearing the output first: cell x owns its
// natural pull sources (x - c_i, i) (with periodic wrap, every element of the
// box has one owner) and writes each one's value or zero, except an element a
// fluid cell bounces into, which that cell writes (non-fluid owners write
// their zeros in a light pass of their own).  Solid and inlet
// outputs do not depend on the state.  Ghost,
// outflow and Neumann cells copy a source cell (their own, the x - 1
// neighbour, the inward neighbour) through a collision with zero relaxation,
// the identity: a second pass adds their output adjoints to the source
// elements with atomic adds, since a fluid cell may pull the same element.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/cslbm.h"
#include "cm_adjoint.hpp"
#include "cm_collide.hpp"
#include "exchange.hpp"
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
    const uint8_t* flags;    // cell kinds or null (fully periodic level)
    const uint32_t* links;   // bounce-back masks of near-wall cells or null
    int nx, ny, nz, periodic;
    int64_t plane;
    AdjointParams ap;
};

// Bounce-back mask of a near-wall cell from its neighbours' kinds (bit i:
// the pull source x - c_i is solid or outside a non-periodic face), as the
// forward step computes it when the level has no links array.
__device__ __forceinline__ uint32_t adj_links(const AdjArgs& a, int x, int y, int z,
                                              const int (&sx)[3], const int (&sy)[3],
                                              const int (&sz)[3])
{
    uint32_t m = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
        if (leaves_box(x, y, z, kCx[i], kCy[i], kCz[i], a.nx, a.ny, a.nz, a.periodic) ||
            (a.flags[src] & kKindMask) == kSolid)
            m |= 1u << i;
    }
    return m;
}

// Zero the owned elements (natural pull sources) of cell (x, y, z) along the
// velocities in dirs that no fluid cell pulls.  The owner x does not pull
// element (x - c_i, i) along these velocities; the only other possible
// reader is the cell x - c_i itself, by bouncing back along -c_i: it does so
// exactly when it is fluid and that link is blocked, i.e. x is solid or the
// link crosses a non-periodic face (the bounce-back masks are prepared from
// the same kinds).  A cell with no fluid neighbour (near_fluid false) zeroes
// its elements unchecked.  D3Q7 direction i is D3Q27 velocity i, with the
// same element positions.
template <bool kScalar>
__device__ __forceinline__ void zero_unpulled(const AdjArgs& a, int x, int y, int z,
                                              const int (&sx)[3], const int (&sy)[3],
                                              const int (&sz)[3], uint32_t dirs, bool solid,
                                              bool near_fluid)
{
    const int64_t P = a.plane;
    if (near_fluid) {
        // every neighbour's kind loaded at once, then the bounced elements masked out
        uint32_t theirs = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
            const bool blocked =
                solid || leaves_box(x, y, z, kCx[i], kCy[i], kCz[i], a.nx, a.ny, a.nz, a.periodic);
            const bool fluid = (a.flags[src] & kKindMask) == kFluid;
            theirs |= (blocked && fluid) ? (1u << i) : 0u;
        }
        dirs &= ~theirs;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!(dirs & (1u << i))) continue;
        const int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
        __builtin_nontemporal_store(0.0f, a.lam0 + i * P + src);
    }
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            if (!(dirs & (1u << i))) continue;
            const int src = sx[kSx[i] + 1] + sy[kSy[i] + 1] + sz[kSz[i] + 1];
            a.mu0[i * P + src] = 0.0f;
        }
    }
}

// cell offsets of the x, y, z neighbours (+1, 0, -1 along each axis, periodic
// wrap): the pull source x - c_i is sx[cx + 1] + sy[cy + 1] + sz[cz + 1]
__device__ __forceinline__ void neighbour_offsets(int x, int y, int z, int nx, int ny, int nz,
                                                  int (&sx)[3], int (&sy)[3], int (&sz)[3])
{
    const int nxy = nx * ny;
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    sx[0] = xp;
    sx[1] = x;
    sx[2] = xm;
    sy[0] = yp * nx;
    sy[1] = y * nx;
    sy[2] = ym * nx;
    sz[0] = zp * nxy;
    sz[1] = z * nxy;
    sz[2] = zm * nxy;
}

template <typename T, bool kScalar, bool kFlags>
__device__ __forceinline__ void adjoint_cell(const AdjArgs& a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz, nxy = nx * ny;
    const int cell = x + nx * y + nxy * z;
    const int64_t P = a.plane;
    int sx[3], sy[3], sz[3];
    neighbour_offsets(x, y, z, nx, ny, nz, sx, sy, sz);
    const T* f = static_cast<const T*>(a.f);
    uint32_t links = 0;
    if (kFlags) {
        const uint8_t flag = a.flags[cell];
        // other kinds: k_adjoint_zeros writes their owned elements, the copy
        // pass adds the outputs of copying kinds
        if ((flag & kKindMask) != kFluid) return;
        if (flag & kNearWall) {
            links = a.links ? a.links[cell] : adj_links(a, x, y, z, sx, sy, sz);
            // a blocked link of a fluid cell hands its element to the
            // neighbour only across a non-periodic face
            const bool on_face = (!(a.periodic & 1) && (x == 0 || x == nx - 1)) ||
                                 (!(a.periodic & 2) && (y == 0 || y == ny - 1)) ||
                                 (!(a.periodic & 4) && (z == 0 || z == nz - 1));
            zero_unpulled<kScalar>(a, x, y, z, sx, sy, sz, links, false, on_face);
        }
    }
    // pull source of velocity i: (plane, cell) as in the forward step
    auto source = [&](int i, int& pl) {
        pl = i;
        int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
        if (kFlags && (links & (1u << i))) {
            src = cell;
            pl = opposite(i);
        }
        return src;
    };
    auto scalar_source = [&](int i, int& pl) {
        pl = i;
        int src = sx[kSx[i] + 1] + sy[kSy[i] + 1] + sz[kSz[i] + 1];
        if (kFlags && (links & (1u << i))) {   // D3Q7 direction i is D3Q27 velocity i
            src = cell;
            pl = scalar_opposite(i);
        }
        return src;
    };

    float h[27], lam[27];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int pl;
        const int src = source(i, pl);
        h[tensor_slot(i)] = Io<T>::ld(f + pl * P + src);
        lam[tensor_slot(i)] = a.lam1[i * P + cell];
    }
    float gv[QS] = {0, 0, 0, 0, 0, 0, 0}, mu[QS] = {0, 0, 0, 0, 0, 0, 0};
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            int pl;
            const int src = scalar_source(i, pl);
            gv[i] = a.g[pl * P + src];
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
    // The 27 pull sources are formed again for the stores instead of kept
    // live through the collision adjoint (54 registers): the empty asm
    // statements hide that the link mask and the neighbour offsets are
    // unchanged.  With them every variant fits two waves per SIMD unspilled.
    if (kFlags) asm volatile("" : "+v"(links));
    asm volatile("" : "+v"(sx[0]), "+v"(sx[1]), "+v"(sx[2]), "+v"(sy[0]), "+v"(sy[1]), "+v"(sy[2]),
                 "+v"(sz[0]), "+v"(sz[1]), "+v"(sz[2]));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int pl;
        const int src = source(i, pl);
        __builtin_nontemporal_store(hb[tensor_slot(i)], a.lam0 + pl * P + src);
    }
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            int pl;
            const int src = scalar_source(i, pl);
            a.mu0[pl * P + src] = gb[i];
        }
    }
    if (a.dtheta) {
        a.dtheta[cell] += thb[0];
        a.dtheta[P + cell] += thb[1];
        a.dtheta[2 * P + cell] += thb[2];
    }
}

// One thread per cell: the adjoint of its update, written to its pull
// sources.  Two waves per SIMD (239-252 VGPRs, no scratch): the second wave
// hides the memory latency of the first.
template <typename T, bool kScalar, bool kFlags>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_adjoint(const AdjArgs a)
{
    adjoint_cell<T, kScalar, kFlags>(a);
}

// Levels with cell kinds, before the fluid pass: the owned elements of the
// non-fluid cells (no fluid cell pulls them except by bouncing into them).
// A pass of its own at full occupancy: in the fluid pass, whose registers
// allow two waves per SIMD, the stores of mostly solid boxes ran slowly.
template <bool kScalar>
__global__ void __launch_bounds__(256) k_adjoint_zeros(const AdjArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int cell = x + a.nx * (y + a.ny * z);
    const uint8_t flag = a.flags[cell];
    const int kind = flag & kKindMask;
    if (kind == kFluid) return;
    int sx[3], sy[3], sz[3];
    neighbour_offsets(x, y, z, a.nx, a.ny, a.nz, sx, sy, sz);
    zero_unpulled<kScalar>(a, x, y, z, sx, sy, sz, ~0u, kind == kSolid, (flag & CSLBM_NEAR_FLUID) != 0);
}

// Second pass on levels with cell kinds: ghost, outflow and Neumann cells
// copy their source cell's state (identity Jacobian), so their output
// adjoints are added to the source elements.
__global__ void __launch_bounds__(256) k_adjoint_copies(const AdjArgs a, bool scalar)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nxy = nx * ny;
    const int cell = x + nx * y + nxy * z;
    const int kind = a.flags[cell] & kKindMask;
    int from;
    if (kind == kGhost) {
        from = cell;
    } else if (kind == kOutflow) {
        from = (x > 0 || (a.periodic & 1)) ? ((x == 0 ? nx - 1 : x - 1) + nx * y + nxy * z) : cell;
    } else if (kind == kNeumann) {
        int xi = x, yi = y, zi = z;
        if (!(a.periodic & 1) && nx > 1) xi = (x == 0) ? 1 : (x == nx - 1 ? nx - 2 : x);
        if (!(a.periodic & 2) && ny > 1) yi = (y == 0) ? 1 : (y == ny - 1 ? ny - 2 : y);
        if (!(a.periodic & 4) && a.nz > 1) zi = (z == 0) ? 1 : (z == a.nz - 1 ? a.nz - 2 : z);
        from = xi + nx * (yi + ny * zi);
    } else {
        return;
    }
    const int64_t P = a.plane;
    // every value loaded before the first atomic: a load-wait-atomic chain
    // per element (the wait covers the previous atomic as well) made each
    // copying wave 2 x 34 memory round trips long
    float l1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) l1[i] = a.lam1[i * P + cell];
#pragma unroll
    for (int i = 0; i < Q; ++i) atomicAdd(a.lam0 + i * P + from, l1[i]);
    if (scalar) {
        float m1[QS];
#pragma unroll
        for (int i = 0; i < QS; ++i) m1[i] = a.mu1[i * P + cell];
#pragma unroll
        for (int i = 0; i < QS; ++i) atomicAdd(a.mu0 + i * P + from, m1[i]);
    }
}

// zero elements n .. plane - 1 of each of the planes
__global__ void __launch_bounds__(256) k_zero_tail(float* p, int planes, int64_t n, int64_t plane)
{
    const int64_t tail = plane - n;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < planes * tail) p[(i / tail) * plane + n + i % tail] = 0.0f;
}

template <typename T>
static void launch_adjoint(const AdjArgs& a, bool scalar, hipStream_t st)
{
    const dim3 block = step_block(a.nx);
    const dim3 grid((a.nx + block.x - 1) / block.x, (a.ny + block.y - 1) / block.y, a.nz);
    if (a.flags) {
        // the fluid pass writes every element of the box; the plane padding
        // beyond it is cleared here
        const int64_t n = (int64_t)a.nx * a.ny * a.nz, tail = a.plane - n;
        if (tail > 0) {
            hipLaunchKernelGGL(k_zero_tail, dim3((unsigned)((Q * tail + 255) / 256)), dim3(256), 0, st,
                               a.lam0, Q, n, a.plane);
            if (scalar)
                hipLaunchKernelGGL(k_zero_tail, dim3((unsigned)((QS * tail + 255) / 256)), dim3(256), 0,
                                   st, a.mu0, QS, n, a.plane);
        }
        if (scalar)
            hipLaunchKernelGGL(k_adjoint_zeros<true>, grid, block, 0, st, a);
        else
            hipLaunchKernelGGL(k_adjoint_zeros<false>, grid, block, 0, st, a);
        if (scalar)
            hipLaunchKernelGGL((k_adjoint<T, true, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_adjoint<T, false, true>), grid, block, 0, st, a);
        hipLaunchKernelGGL(k_adjoint_copies, grid, block, 0, st, a, scalar);
        return;
    }
    if (scalar)
        hipLaunchKernelGGL((k_adjoint<T, true, false>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_adjoint<T, false, false>), grid, block, 0, st, a);
}

int launch_adjoint_into(const cslbm_level* L, const void* fin, const float* gin,
                        const float* lam_next, const float* mu_next, float* lam, float* mu,
                        float* dtheta, hipStream_t stream)
{
    const bool scalar = gin != nullptr;
    AdjArgs a;
    a.f = fin;
    a.g = gin;
    a.theta = L->force;
    a.lam1 = lam_next;
    a.mu1 = scalar ? mu_next : nullptr;
    a.lam0 = lam;
    a.mu0 = scalar ? mu : nullptr;
    a.dtheta = dtheta;
    a.flags = L->flags;
    a.links = L->links;
    a.nx = L->nx;
    a.ny = L->ny;
    a.nz = L->nz;
    a.periodic = L->periodic & 7;
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
    if ((L->periodic & 7) != 7 && !L->flags)
        return fail(CSLBM_ERR_UNSUPPORTED,
                    "the adjoint step of a level without cell flags needs a fully periodic box");
    if (L->p.grad_mode != 0)
        return fail(CSLBM_ERR_UNSUPPORTED,
                    "the adjoint step differentiates the local gradient estimate (grad_mode 0)");
    if (L->brick_table) return fail(CSLBM_ERR_UNSUPPORTED, "the adjoint of a brick level");
    if (L->wall_cells != 0)
        return fail(CSLBM_ERR_UNSUPPORTED, "the adjoint does not differentiate wall nodes");
    if (!lam_next || !lam) return fail(CSLBM_ERR_ARG, "adjoint buffers are NULL");
    if (lam_next == lam) return fail(CSLBM_ERR_ARG, "lam and lam_next alias");
    const bool scalar = L->g != nullptr;
    if (scalar && (!mu_next || !mu || mu == mu_next))
        return fail(CSLBM_ERR_ARG, "a level with a scalar needs distinct mu and mu_next");
    return launch_adjoint_into(L, L->f, L->g, lam_next, mu_next, lam, mu, dtheta, stream);
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
