// step.hip -- the hot path of libcslbm (gfx950): k_step, the fused pull-stream
// + central-moment collision (one thread per cell, x fastest so that a
// wave64 covers 64 consecutive cells of a row: every one of the 27 plane
// loads and 27 plane stores of a wave is a contiguous 256-byte (FP32) or
// 128-byte (FP16) segment), and its host-side launchers.  It is bound by HBM
// bandwidth: 27 reads + 27 writes per lattice update and nothing else.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "../../include/cslbm.h"
#include "brick.hpp"
#include "cm_collide.hpp"
#include "internal.hpp"
#include "lattice.hpp"
#include "wall.hpp"

namespace cslbm {

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------
struct StepArgs {
    const void* f;
    void* fo;
    const float* g;
    float* go;
    const uint8_t* flags;
    const uint32_t* links;
    const float* force;
    int nx, ny, nz, periodic;
    int64_t plane;
    Rates r;
    float beta, s_ref, inv_tau_s;
    float u_in[3];
    float s_in;
    // fused quadratic time interpolation of the output (finer scales):
    // out = l0 * t0 + l1 * f + l2 * step(f), t0 the state at t_n
    const void* t0;
    const float* gt0;
    float l0, l1, l2;
    // finite-difference gradient mode: stored velocity [3][N] of the input
    // state and of the output state
    const float* vel;
    float* vel_out;
    int64_t ncells;
    const float* gmax;    // running maximum of the gradient field, or null
    BrickMap bricks;      // sparse brick storage (table null: dense box)
};

// |grad u|_F at cell (x, y, z) of a stored velocity field [3][N] by central
// differences with periodic wrap (the one formula of the gradient mode:
// the step and the field maximum both use it, so they agree bit for bit).
__device__ __forceinline__ float grad_fd(const float* vel, int64_t Nc, int x, int y, int z, int nx,
                                         int ny, int nz)
{
    const int nxy = nx * ny;
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int row = nx * y + nxy * z;
    const int cxm = xm + row, cxp = xp + row;
    const int cym = x + nx * ym + nxy * z, cyp = x + nx * yp + nxy * z;
    const int czm = x + nx * y + nxy * zm, czp = x + nx * y + nxy * zp;
    float sum = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float* U = vel + b * Nc;
        const float dx = 0.5f * (U[cxp] - U[cxm]);
        const float dy = 0.5f * (U[cyp] - U[cym]);
        const float dz = 0.5f * (U[czp] - U[czm]);
        sum += dx * dx + dy * dy + dz * dz;
    }
    return sqrtf(sum);
}

// Output store of k_step: the new state, or (kTime) its quadratic time
// interpolation l0 * t0 + l1 * (input state) + l2 * (new state) at the cell.
template <typename T, bool kTime>
__device__ __forceinline__ void store_out(const StepArgs& a, T* fo, int64_t e, float v)
{
    if (kTime) {
        const float x0 = Io<T>::ld(static_cast<const T*>(a.t0) + e);
        const float x1 = Io<T>::ld(static_cast<const T*>(a.f) + e);
        v = a.l0 * x0 + a.l1 * x1 + a.l2 * v;
    }
    Io<T>::st(fo + e, v);
}

template <bool kTime>
__device__ __forceinline__ void store_gout(const StepArgs& a, int64_t e, float v)
{
    if (kTime) v = a.l0 * a.gt0[e] + a.l1 * a.g[e] + a.l2 * v;
    __builtin_nontemporal_store(v, a.go + e);
}

// Element `idx` of one plane addressed as uniform base + 32-bit byte offset.
// Used for binary16 planes only: cells are validated below 2^31, so the byte
// offset idx * 2 always fits in 32 bits.
template <typename T>
__device__ __forceinline__ T* plane_at(T* base, int idx)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + (uint32_t)idx * (uint32_t)sizeof(T));
}

// Copy source of a Neumann (zero normal gradient) far-field cell: one cell
// inward along every non-periodic face the cell lies on.
__device__ __forceinline__ int inward_cell(const StepArgs& a, int x, int y, int z)
{
    if (!(a.periodic & 1) && a.nx > 1) x = (x == 0) ? 1 : (x == a.nx - 1 ? a.nx - 2 : x);
    if (!(a.periodic & 2) && a.ny > 1) y = (y == 0) ? 1 : (y == a.ny - 1 ? a.ny - 2 : y);
    if (!(a.periodic & 4) && a.nz > 1) z = (z == 0) ? 1 : (z == a.nz - 1 ? a.nz - 2 : z);
    return x + a.nx * (y + a.ny * z);
}

// Bounce-back mask of a near-wall cell computed from the neighbours' kinds
// (used only when the level has no precomputed links array): bit i is set
// when the pull source x - c_i is solid or outside a non-periodic face.
__device__ __forceinline__ uint32_t bounce_links(const StepArgs& a, int x, int y, int z,
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

// Brick levels: the block's brick and its 26 neighbours (index -1: not
// stored or outside the box) are read once into LDS; the pull source of
// velocity i of the cell at brick-local (lx, ly, lz) is then the
// neighbouring brick's cell at (lx - cx, ly - cy, lz - cz) mod 8, or the
// cell itself when that brick is not stored (a valid brick level gives no
// fluid cell such a source).
__device__ __forceinline__ int brick_source(const int* nbr, int c, int cx, int cy, int cz)
{
    const int lx = (c & 7) - cx, ly = ((c >> 3) & 7) - cy, lz = ((c >> 6) & 7) - cz;
    const int k = (lx < 0 ? 0 : (lx > 7 ? 2 : 1)) + 3 * (ly < 0 ? 0 : (ly > 7 ? 2 : 1)) +
                  9 * (lz < 0 ? 0 : (lz > 7 ? 2 : 1));
    const int b = nbr[k];
    return b < 0 ? c : (b << 9) + (lx & 7) + ((ly & 7) << 3) + ((lz & 7) << 6);
}

// bounce-back mask from the neighbours' kinds (a source that is not stored
// counts as a wall)
__device__ __forceinline__ uint32_t bounce_links_brick(const StepArgs& a, const int* nbr, int c)
{
    uint32_t m = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int s = brick_source(nbr, c, kCx[i], kCy[i], kCz[i]);
        if (s == c || (a.flags[s] & kKindMask) == kSolid) m |= 1u << i;
    }
    return m;
}

// ---------------------------------------------------------------------------
// K: fused pull-stream + collide
// ---------------------------------------------------------------------------
template <typename T, bool kFlags, bool kForce, bool kScalar, bool kTime, bool kGradFD,
          bool kBrick = false>
__global__ void __launch_bounds__(256) k_step(const StepArgs a)
{
    // dense box: (x, y, z) from the 3-D grid; brick level: two blocks per
    // stored brick, each 256 cells of it in storage order
    int x, y, z, cell;
    __shared__ int nbr[kBrick ? 27 : 1];
    if (kBrick) {
        const int b = blockIdx.x >> 1;
        cell = (b << 9) + threadIdx.x + ((blockIdx.x & 1) << 8);
        brick_xyz(a.bricks, cell, x, y, z);
        if (threadIdx.x < 27) {
            const int t = threadIdx.x;
            const int bx = a.bricks.origin[3 * b] + t % 3 - 1;
            const int by = a.bricks.origin[3 * b + 1] + (t / 3) % 3 - 1;
            const int bz = a.bricks.origin[3 * b + 2] + t / 9 - 1;
            const bool in = bx >= 0 && by >= 0 && bz >= 0 && bx < a.bricks.bnx && by < a.bricks.bny &&
                            bz < a.bricks.bnz;
            nbr[t] = in ? a.bricks.table[bx + a.bricks.bnx * (by + a.bricks.bny * bz)] : -1;
        }
        __syncthreads();
    } else {
        x = blockIdx.x * blockDim.x + threadIdx.x;
        y = blockIdx.y * blockDim.y + threadIdx.y;
        z = blockIdx.z;
        if (x >= a.nx || y >= a.ny) return;
        cell = x + a.nx * y + a.nx * a.ny * z;
    }
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    const int64_t P = a.plane;
    const T* __restrict__ f = static_cast<const T*>(a.f);
    T* __restrict__ fo = static_cast<T*>(a.fo);
    constexpr bool kOff32 = sizeof(T) == 2;

    // source coordinates of the pull, indexed by (c + 1): c = -1 pulls from
    // x + 1, c = +1 from x - 1 (periodic wrap; links that leave the box
    // through a non-periodic face are in the cell's bounce-back mask)
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1;
    const int zp = (z == nz - 1) ? 0 : z + 1;
    const int sx[3] = {xp, x, xm};
    const int sy[3] = {yp * nx, y * nx, ym * nx};
    const int sz[3] = {zp * nxy, z * nxy, zm * nxy};

    // Cell kinds without divergent code paths: every lane issues the same
    // 27 (+7) loads and stores with its own addresses.  Fluid cells pull
    // (bounce-back links from the per-cell mask), ghost, outflow and Neumann
    // cells load their copy source, solid and inlet cells read their own
    // cell and discard it; the
    // collision runs with zero relaxation on non-fluid lanes (an identity
    // up to rounding), and inlet lanes start from the inlet equilibrium.
    int kind = kFluid;
    uint32_t links = 0;
    int from = cell;
    int wall_code = 0;
    if (kFlags) {
        const uint8_t flag = a.flags[cell];
        kind = flag & kKindMask;
        wall_code = flag >> kWallNormalShift;
        if (kBrick) {
            if (flag & kNearWall) links = a.links ? a.links[cell] : bounce_links_brick(a, nbr, cell);
            if (kind == kOutflow) from = brick_source(nbr, cell, 1, 0, 0);
            if (kind == kNeumann) {
                int xi = x, yi = y, zi = z;   // no periodic axis on a brick level
                if (nx > 1) xi = (x == 0) ? 1 : (x == nx - 1 ? nx - 2 : x);
                if (ny > 1) yi = (y == 0) ? 1 : (y == ny - 1 ? ny - 2 : y);
                if (nz > 1) zi = (z == 0) ? 1 : (z == nz - 1 ? nz - 2 : z);
                const int s = brick_cell(a.bricks, xi, yi, zi);
                from = s < 0 ? cell : s;
            }
        } else {
            if (flag & kNearWall) links = a.links ? a.links[cell] : bounce_links(a, x, y, z, sx, sy, sz);
            if (kind == kOutflow && (x > 0 || (a.periodic & 1))) from = xm + nx * y + nxy * z;
            if (kind == kNeumann) from = inward_cell(a, x, y, z);
        }
    }
    // wall nodes pull and collide like fluid nodes (their populations are
    // rebuilt in between)
    const bool fluid = kind == kFluid || kind == kWall;
    const bool copies = kind == kGhost || kind == kOutflow || kind == kNeumann;
    const bool loads = fluid || copies;

    float v[27];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int src = kBrick ? brick_source(nbr, cell, kCx[i], kCy[i], kCz[i])
                         : sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
        int pl = i;
        if (kFlags) {
            if (links & (1u << i)) {   // halfway bounce-back: own opposite population
                src = cell;
                pl = opposite(i);
            }
            if (!fluid) {   // copy source; solid and inlet lanes read their own cell
                src = from;
                pl = i;
            }
        }
        // unconditional: no branch.  Without flags the plane base is uniform
        // and the binary16 kernel addresses it with a 32-bit lane offset
        // (measured faster there; the FP32 kernel is faster as written).
        const float hv = (kOff32 && !kFlags) ? Io<T>::ld(plane_at(f + i * P, src))
                                             : Io<T>::ld(f + pl * P + src);
        v[tensor_slot(i)] = (!kFlags || loads) ? hv : 0.0f;
    }
    if (kFlags && kind == kInlet) shifted_equilibrium(v, 1.0f, a.u_in[0], a.u_in[1], a.u_in[2]);

    float gv[QS];
    float s = 0.0f;
    if (kScalar) {
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            int src = kBrick ? brick_source(nbr, cell, kSx[i], kSy[i], kSz[i])
                             : sx[kSx[i] + 1] + sy[kSy[i] + 1] + sz[kSz[i] + 1];
            int pl = i;
            if (kFlags) {
                if (links & (1u << i)) {   // D3Q7 direction i is D3Q27 velocity i
                    src = cell;
                    pl = scalar_opposite(i);
                }
                if (!fluid) {
                    src = from;
                    pl = i;
                }
            }
            const float gl = a.g[pl * P + src];
            gv[i] = (!kFlags || loads) ? gl : 0.0f;
        }
        s = (gv[0] + (gv[1] + gv[2])) + ((gv[3] + gv[4]) + (gv[5] + gv[6]));
    }

    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    if (kForce && fluid) {
        Fx = a.force[cell];
        Fy = a.force[P + cell];
        Fz = a.force[2 * P + cell];
    }
    if (kScalar && fluid) Fz += a.beta * (s - a.s_ref);
    if (kFlags && kind == kWall) {
        if (wall_code >= 1 && wall_code <= 6)
            wall_regularize(v, wall_code, Fx, Fy, Fz);
        else   // not on one flat axis-aligned wall: flag the cell with NaN
            v[13] = __builtin_nanf("");
    }

    // gradient mode: |grad u|_F of the stored velocity field by central
    // differences (the level is fully periodic: kGradFD excludes flags)
    float g_given = -1.0f;
    Rates rates = a.r;
    if (kGradFD) {
        g_given = grad_fd(a.vel, a.ncells, x, y, z, nx, ny, nz);
        if (a.gmax) {   // running maximum: normalise by the field's largest gradient
            const float gm = *a.gmax;
            rates.inv_gmax = gm > 0.0f ? 1.0f / gm : 0.0f;
        }
    }
    const CellMacro mc = cm_collide(v, rates, Fx, Fy, Fz, fluid, g_given);
    if (kGradFD) {
        // velocity of the new state as read back from it: (j~ - F/2)/rho
        // equals the collision velocity (j + F/2)/rho since j~ = j + F
        a.vel_out[cell] = mc.ux;
        a.vel_out[a.ncells + cell] = mc.uy;
        a.vel_out[2 * a.ncells + cell] = mc.uz;
    }

#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (kOff32 && !kTime) {
            // the plane base stays a uniform SGPR pair, so every store is
            // base + the one 32-bit lane offset; without the empty asm the
            // compiler chains 64-bit VALU adds from plane to plane
            using G16 = __attribute__((address_space(1))) _Float16;
            G16* base = (G16*)(fo + i * P);
            asm("" : "+s"(base));
            G16* p = (G16*)((__attribute__((address_space(1))) char*)base + (uint32_t)cell * 2u);
            __builtin_nontemporal_store(static_cast<_Float16>(v[tensor_slot(i)]), p);
        } else
            store_out<T, kTime>(a, fo, i * P + cell, v[tensor_slot(i)]);
    }

    if (kScalar) {
        const float ux = kind == kInlet ? a.u_in[0] : mc.ux;
        const float uy = kind == kInlet ? a.u_in[1] : mc.uy;
        const float uz = kind == kInlet ? a.u_in[2] : mc.uz;
        const float sc = kind == kInlet ? a.s_in : s;
        // fluid and wall: BGK; inlet: equilibrium; ghost/outflow: copy; solid: 0
        const float relax = fluid ? a.inv_tau_s : (kind == kInlet ? 1.0f : 0.0f);
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const float ge = scalar_eq(i, sc, ux, uy, uz);
            store_gout<kTime>(a, i * P + cell, gv[i] - (gv[i] - ge) * relax);
        }
    }
}

// Field maximum of the gradient-mode G.  One thread per cell in the step's
// launch shape; every block reduces its maximum in LDS (out-of-box threads
// take part with 0) and folds it into one of the partial slots with an
// atomic maximum on the bit pattern (G >= 0, so the order of float bit
// patterns is the order of the values and the result does not depend on
// the order of the atomics).  The final pass reduces the slots, stores the
// maximum and clears the slots for the next step.
constexpr int kGmaxBlocks = CSLBM_GMAX_BUF - 1;

__global__ void __launch_bounds__(256) k_grad_max_partials(const float* vel, int nx, int ny, int nz,
                                                           unsigned int* slots)
{
    __shared__ float red[256];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int64_t N = (int64_t)nx * ny * nz;
    red[tid] = (x < nx && y < ny) ? grad_fd(vel, N, x, y, z, nx, ny, nz) : 0.0f;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        const unsigned int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        atomicMax(slots + (b % kGmaxBlocks), __float_as_uint(red[0]));
    }
}

__global__ void __launch_bounds__(256) k_grad_max_final(float* buf)
{
    __shared__ float red[256];
    unsigned int* slots = reinterpret_cast<unsigned int*>(buf);
    float m = 0.0f;
    for (int i = threadIdx.x; i < kGmaxBlocks; i += blockDim.x) {
        m = fmaxf(m, __uint_as_float(slots[i]));
        slots[i] = 0u;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) buf[kGmaxBlocks] = red[0];
}

dim3 step_block(int nx)
{
    int best = 256;
    int64_t best_pad = ((nx + 255) / 256) * 256 - nx;
    for (int bx : {128, 64}) {
        const int64_t pad = ((int64_t)(nx + bx - 1) / bx) * bx - nx;
        if (pad < best_pad) {
            best = bx;
            best_pad = pad;
        }
    }
    return dim3(best, 256 / best, 1);
}

template <typename T, bool kFlags, bool kForce, bool kScalar, bool kTime = false,
          bool kGradFD = false>
static void launch_step(const StepArgs& a, hipStream_t st)
{
    const dim3 block = step_block(a.nx);
    const dim3 grid((a.nx + block.x - 1) / block.x, (a.ny + block.y - 1) / block.y, a.nz);
    hipLaunchKernelGGL((k_step<T, kFlags, kForce, kScalar, kTime, kGradFD>), grid, block, 0, st, a);
}

// brick levels: flags, no force field, two 256-thread blocks per stored brick
template <typename T>
static void launch_step_brick(const StepArgs& a, bool scalar, bool time, int n_bricks, hipStream_t st)
{
    const dim3 grid(2u * (unsigned)n_bricks), block(256);
    if (scalar && time)
        hipLaunchKernelGGL((k_step<T, true, false, true, true, false, true>), grid, block, 0, st, a);
    else if (scalar)
        hipLaunchKernelGGL((k_step<T, true, false, true, false, false, true>), grid, block, 0, st, a);
    else if (time)
        hipLaunchKernelGGL((k_step<T, true, false, false, true, false, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_step<T, true, false, false, false, false, true>), grid, block, 0, st, a);
}

// gradient-mode variants: fully periodic levels without flags
template <typename T>
static void dispatch_step_grad(const StepArgs& a, bool force, bool scalar, hipStream_t st)
{
    const int key = (force ? 2 : 0) | (scalar ? 1 : 0);
    switch (key) {
        case 0: launch_step<T, false, false, false, false, true>(a, st); break;
        case 1: launch_step<T, false, false, true, false, true>(a, st); break;
        case 2: launch_step<T, false, true, false, false, true>(a, st); break;
        default: launch_step<T, false, true, true, false, true>(a, st); break;
    }
}

// time-interpolating variants exist for flagged levels only (finer scales)
template <typename T>
static void dispatch_step(const StepArgs& a, bool flags, bool force, bool scalar, bool time,
                          hipStream_t st)
{
    if (time) {
        const int key = (force ? 2 : 0) | (scalar ? 1 : 0);
        switch (key) {
            case 0: launch_step<T, true, false, false, true>(a, st); break;
            case 1: launch_step<T, true, false, true, true>(a, st); break;
            case 2: launch_step<T, true, true, false, true>(a, st); break;
            default: launch_step<T, true, true, true, true>(a, st); break;
        }
        return;
    }
    const int key = (flags ? 4 : 0) | (force ? 2 : 0) | (scalar ? 1 : 0);
    switch (key) {
        case 0: launch_step<T, false, false, false>(a, st); break;
        case 1: launch_step<T, false, false, true>(a, st); break;
        case 2: launch_step<T, false, true, false>(a, st); break;
        case 3: launch_step<T, false, true, true>(a, st); break;
        case 4: launch_step<T, true, false, false>(a, st); break;
        case 5: launch_step<T, true, false, true>(a, st); break;
        case 6: launch_step<T, true, true, false>(a, st); break;
        default: launch_step<T, true, true, true>(a, st); break;
    }
}

int launch_step_into(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                     float* gout, hipStream_t stream)
{
    return launch_step_interp(L, fin, fout, gin, gout, nullptr, nullptr, 0.0, 0.0, 1.0, stream);
}

static StepArgs step_args(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                          float* gout)
{
    StepArgs a;
    a.t0 = nullptr;
    a.gt0 = nullptr;
    a.l0 = 0.0f;
    a.l1 = 0.0f;
    a.l2 = 1.0f;
    a.vel = nullptr;
    a.vel_out = nullptr;
    a.ncells = 0;
    a.gmax = nullptr;
    a.f = fin;
    a.fo = fout;
    a.g = gin;
    a.go = gout;
    a.flags = L->flags;
    a.links = L->links;
    a.force = L->force;
    a.nx = L->nx;
    a.ny = L->ny;
    a.nz = L->nz;
    a.periodic = L->periodic & 7;
    a.plane = L->plane;
    a.r = make_rates(L->p);
    a.beta = (float)L->p.beta;
    a.s_ref = (float)L->p.s_ref;
    a.inv_tau_s = gin ? (float)(1.0 / L->p.tau_s) : 0.0f;
    for (int k = 0; k < 3; ++k) a.u_in[k] = (float)L->p.u_in[k];
    a.s_in = (float)L->p.s_in;
    a.bricks = brick_map(L);
    return a;
}

// One step in the finite-difference gradient mode (grad_mode 1): the
// adaptive factor takes |grad u|_F of vel (the input state's velocity) and
// the new state's velocity goes to vel_out.
int launch_step_grad(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                     float* gout, const float* vel, float* vel_out, hipStream_t stream)
{
    StepArgs a = step_args(L, fin, fout, gin, gout);
    a.vel = vel;
    a.vel_out = vel_out;
    a.ncells = cells_of(L);
    if (L->p.gmax_running) {
        const dim3 block = step_block(L->nx);
        const dim3 grid((L->nx + block.x - 1) / block.x, (L->ny + block.y - 1) / block.y, L->nz);
        hipLaunchKernelGGL(k_grad_max_partials, grid, block, 0, stream, vel, L->nx, L->ny, L->nz,
                           reinterpret_cast<unsigned int*>(L->gmax_buf));
        hipLaunchKernelGGL(k_grad_max_final, dim3(1), dim3(256), 0, stream, L->gmax_buf);
        a.gmax = L->gmax_buf + kGmaxBlocks;
    }
    if (L->storage == CSLBM_F32)
        dispatch_step_grad<float>(a, L->force != nullptr, gin != nullptr, stream);
    else
        dispatch_step_grad<_Float16>(a, L->force != nullptr, gin != nullptr, stream);
    return check_launch("k_step");
}

int launch_step_interp(const cslbm_level* L, const void* fin, void* fout, const float* gin,
                       float* gout, const void* t0, const float* gt0, double l0, double l1,
                       double l2, hipStream_t stream)
{
    if (L->p.grad_mode != 0)
        return fail(CSLBM_ERR_UNSUPPORTED,
                    "the finite-difference gradient mode runs through cslbm_step only");
    StepArgs a = step_args(L, fin, fout, gin, gout);
    a.t0 = t0;
    a.gt0 = gt0;
    a.l0 = (float)l0;
    a.l1 = (float)l1;
    a.l2 = (float)l2;
    const bool has_flags = L->flags != nullptr;
    const bool has_force = L->force != nullptr;
    const bool has_scalar = gin != nullptr;
    const bool time = t0 != nullptr;
    if (time && !has_flags)
        return fail(CSLBM_ERR_UNSUPPORTED, "time-interpolating steps need a flagged level");
    if (L->brick_table) {   // validated: flags, no force field
        if (L->storage == CSLBM_F32)
            launch_step_brick<float>(a, has_scalar, time, L->n_bricks, stream);
        else
            launch_step_brick<_Float16>(a, has_scalar, time, L->n_bricks, stream);
        return check_launch("k_step (bricks)");
    }
    if (L->storage == CSLBM_F32)
        dispatch_step<float>(a, has_flags, has_force, has_scalar, time, stream);
    else
        dispatch_step<_Float16>(a, has_flags, has_force, has_scalar, time, stream);
    return check_launch("k_step");
}

}  // namespace cslbm
