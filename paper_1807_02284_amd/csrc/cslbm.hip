// cslbm.hip -- single-level kernels and the C ABI of libcslbm (gfx950).
//
// Hot path: k_step, the fused pull-stream + central-moment collision (one
// thread per cell, x fastest so that a wave64 covers 64 consecutive cells of
// a row: every one of the 27 plane loads and 27 plane stores of a wave is a
// contiguous 256-byte (FP32) or 128-byte (FP16) segment).  It is bound by
// HBM bandwidth: 27 reads + 27 writes per lattice update and nothing else.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>

#include "../../include/cslbm.h"
#include "cm_collide.hpp"
#include "internal.hpp"
#include "lattice.hpp"

namespace cslbm {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int check_launch(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CSLBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return CSLBM_OK;
}

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

// D3Q7 equilibrium g^eq_i = w_i s (1 + 4 c_i.u)  (cs^2 = 1/4)
__device__ __forceinline__ float scalar_eq(int i, float s, float ux, float uy, float uz)
{
    return kSw[i] * s * (1.0f + 4.0f * (kSx[i] * ux + kSy[i] * uy + kSz[i] * uz));
}

__device__ __forceinline__ bool leaves_box(int x, int y, int z, int cx, int cy, int cz, int nx,
                                           int ny, int nz, int periodic)
{
    // the pull source x - c lies outside a non-periodic face
    const bool ox = !(periodic & 1) && ((cx == 1 && x == 0) || (cx == -1 && x == nx - 1));
    const bool oy = !(periodic & 2) && ((cy == 1 && y == 0) || (cy == -1 && y == ny - 1));
    const bool oz = !(periodic & 4) && ((cz == 1 && z == 0) || (cz == -1 && z == nz - 1));
    return ox || oy || oz;
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

// ---------------------------------------------------------------------------
// K: fused pull-stream + collide
// ---------------------------------------------------------------------------
template <typename T, bool kFlags, bool kForce, bool kScalar, bool kTime, bool kGradFD>
__global__ void __launch_bounds__(256) k_step(const StepArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    const int cell = x + nx * y + nxy * z;
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
    if (kFlags) {
        const uint8_t flag = a.flags[cell];
        kind = flag & kKindMask;
        if (flag & kNearWall) links = a.links ? a.links[cell] : bounce_links(a, x, y, z, sx, sy, sz);
        if (kind == kOutflow && (x > 0 || (a.periodic & 1))) from = xm + nx * y + nxy * z;
        if (kind == kNeumann) from = inward_cell(a, x, y, z);
    }
    const bool fluid = kind == kFluid;
    const bool copies = kind == kGhost || kind == kOutflow || kind == kNeumann;
    const bool loads = fluid || copies;

    float v[27];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int src = sx[kCx[i] + 1] + sy[kCy[i] + 1] + sz[kCz[i] + 1];
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
            int src = sx[kSx[i] + 1] + sy[kSy[i] + 1] + sz[kSz[i] + 1];
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
        if (kOff32 && !kTime)
            Io<T>::st(plane_at(fo + i * P, cell), v[tensor_slot(i)]);
        else
            store_out<T, kTime>(a, fo, i * P + cell, v[tensor_slot(i)]);
    }

    if (kScalar) {
        const float ux = kind == kInlet ? a.u_in[0] : mc.ux;
        const float uy = kind == kInlet ? a.u_in[1] : mc.uy;
        const float uz = kind == kInlet ? a.u_in[2] : mc.uz;
        const float sc = kind == kInlet ? a.s_in : s;
        // fluid: BGK; inlet: equilibrium; ghost/outflow: copy; solid: 0
        const float relax = kind == kFluid ? a.inv_tau_s : (kind == kInlet ? 1.0f : 0.0f);
#pragma unroll
        for (int i = 0; i < QS; ++i) {
            const float ge = scalar_eq(i, sc, ux, uy, uz);
            store_gout<kTime>(a, i * P + cell, gv[i] - (gv[i] - ge) * relax);
        }
    }
}

// ---------------------------------------------------------------------------
// auxiliary kernels (one thread per cell, 1D launch over N)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cell_coords(int64_t c, int nx, int ny, int& x, int& y, int& z)
{
    x = (int)(c % nx);
    y = (int)((c / nx) % ny);
    z = (int)(c / ((int64_t)nx * ny));
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

__global__ void k_prepare_flags(uint8_t* flags, uint32_t* links, int nx, int ny, int nz,
                                int periodic)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    int x, y, z;
    cell_coords(c, nx, ny, x, y, z);
    const uint8_t kind = flags[c] & kKindMask;
    uint32_t m = 0;
    if (kind == kFluid) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (leaves_box(x, y, z, kCx[i], kCy[i], kCz[i], nx, ny, nz, periodic)) {
                m |= 1u << i;
                continue;
            }
            const int xs = (x - kCx[i] + nx) % nx, ys = (y - kCy[i] + ny) % ny,
                      zs = (z - kCz[i] + nz) % nz;
            if ((flags[xs + (int64_t)nx * (ys + (int64_t)ny * zs)] & kKindMask) == kSolid)
                m |= 1u << i;
        }
    }
    flags[c] = kind | (m ? kNearWall : 0);
    if (links) links[c] = m;
}

template <typename T>
__global__ void k_init_eq(T* f, float* g, int64_t N, int64_t P, const float* rho, const float* u,
                          const float* s)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const float r = rho ? rho[c] : 1.0f;
    const float ux = u[c], uy = u[N + c], uz = u[2 * N + c];
    float v[27];
    shifted_equilibrium(v, r, ux, uy, uz);
#pragma unroll
    for (int i = 0; i < Q; ++i) Io<T>::st(f + i * P + c, v[tensor_slot(i)]);
    if (g) {
        const float sc = s ? s[c] : 0.0f;
#pragma unroll
        for (int i = 0; i < QS; ++i) g[i * P + c] = scalar_eq(i, sc, ux, uy, uz);
    }
}

template <typename T>
__global__ void k_set_pop(T* f, float* g, int64_t N, int64_t P, const float* src, const float* gsrc,
                          int shifted)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float v = src[i * N + c];
        Io<T>::st(f + i * P + c, shifted ? v : v - weight(i));
    }
    if (g && gsrc)
#pragma unroll
        for (int i = 0; i < QS; ++i) g[i * P + c] = gsrc[i * N + c];
}

// Population copy between two levels of one storage type, cell list to
// cell list (the kept part of a rebuilt region).  One thread per cell.
template <typename T>
__global__ void __launch_bounds__(256) k_copy_cells(const T* f, const float* g, int64_t P, T* fo,
                                                    float* go, int64_t Po, const int32_t* src,
                                                    const int32_t* dst, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t a = src[k], b = dst[k];
#pragma unroll
    for (int i = 0; i < Q; ++i) fo[i * Po + b] = f[i * P + a];
    if (g)
#pragma unroll
        for (int i = 0; i < QS; ++i) go[i * Po + b] = g[i * P + a];
}

template <typename T>
__global__ void k_get_pop(const T* f, const float* g, int64_t N, int64_t P, float* dst, float* gdst,
                          int shifted)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float h = Io<T>::ld(f + i * P + c);
        dst[i * N + c] = shifted ? h : h + weight(i);
    }
    if (g && gdst)
#pragma unroll
        for (int i = 0; i < QS; ++i) gdst[i * N + c] = g[i * P + c];
}

template <typename T>
__global__ void k_macro(const T* f, const float* g, const float* force, int64_t N, int64_t P,
                        float beta, float s_ref, float* rho, float* u, float* s)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    float v[27];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[tensor_slot(i)] = Io<T>::ld(f + i * P + c);
    float dr, jx, jy, jz;
    moments0(v, dr, jx, jy, jz);
    float sc = 0.0f;
    if (g)
#pragma unroll
        for (int i = 0; i < QS; ++i) sc += g[i * P + c];
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    if (force) {
        Fx = force[c];
        Fy = force[P + c];
        Fz = force[2 * P + c];
    }
    if (g) Fz += beta * (sc - s_ref);
    const float r = 1.0f + dr;
    if (rho) rho[c] = r;
    if (u) {
        u[c] = (jx - 0.5f * Fx) / r;
        u[N + c] = (jy - 0.5f * Fy) / r;
        u[2 * N + c] = (jz - 0.5f * Fz) / r;
    }
    if (s) s[c] = sc;
}

// |curl u| by central differences of a dense velocity field (periodic wrap on
// periodic axes, one-sided differences at non-periodic faces)
__global__ void __launch_bounds__(256) k_vorticity(const float* u, int nx, int ny, int nz,
                                                   int periodic, float* out, float* speed)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    int x, y, z;
    cell_coords(c, nx, ny, x, y, z);
    const int n[3] = {nx, ny, nz};
    const int p[3] = {x, y, z};
    float grad[3][3];   // grad[a][b] = d u_a / d x_b
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        int lo = p[b] - 1, hi = p[b] + 1;
        float h = 2.0f;
        if (periodic & (1 << b)) {
            lo = (lo + n[b]) % n[b];
            hi = hi % n[b];
        } else {
            if (lo < 0) { lo = 0; h = 1.0f; }
            if (hi >= n[b]) { hi = n[b] - 1; h = 1.0f; }
            if (n[b] == 1) h = 0.0f;
        }
        int ql[3] = {x, y, z}, qh[3] = {x, y, z};
        ql[b] = lo;
        qh[b] = hi;
        const int64_t cl = ql[0] + (int64_t)nx * (ql[1] + (int64_t)ny * ql[2]);
        const int64_t ch = qh[0] + (int64_t)nx * (qh[1] + (int64_t)ny * qh[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            grad[a][b] = h > 0.0f ? (u[a * N + ch] - u[a * N + cl]) / h : 0.0f;
    }
    const float wx = grad[2][1] - grad[1][2], wy = grad[0][2] - grad[2][0], wz = grad[1][0] - grad[0][1];
    out[c] = sqrtf(wx * wx + wy * wy + wz * wz);
    if (speed) {
        const float a = u[c], b = u[N + c], d = u[2 * N + c];
        speed[c] = sqrtf(a * a + b * b + d * d);
    }
}

// FP64 conservation: per-block partial sums (count, sum h, sum c h, sum g),
// then one block adds the partials in a fixed order.
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;
constexpr int kRedVals = 6;

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
    k_conserved_partials(const T* f, const float* g, const uint8_t* flags, int64_t N, int64_t P,
                         double* partials)
{
    double acc[kRedVals] = {0, 0, 0, 0, 0, 0};
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (flags) {
            const int kind = flags[c] & kKindMask;
            if (kind == kSolid || kind == kGhost) continue;
        }
        double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double h = (double)Io<T>::ld(f + i * P + c);
            dr += h;
            jx += kCx[i] * h;
            jy += kCy[i] * h;
            jz += kCz[i] * h;
        }
        double sc = 0.0;
        if (g)
#pragma unroll
            for (int i = 0; i < QS; ++i) sc += (double)g[i * P + c];
        acc[0] += 1.0;
        acc[1] += dr;
        acc[2] += jx;
        acc[3] += jy;
        acc[4] += jz;
        acc[5] += sc;
    }
    __shared__ double sm[kRedVals][kRedThreads];
#pragma unroll
    for (int k = 0; k < kRedVals; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kRedVals; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kRedVals; ++k) partials[blockIdx.x * kRedVals + k] = sm[k][0];
}

__global__ void __launch_bounds__(kRedThreads) k_conserved_final(const double* partials, int nblocks,
                                                                 double* out)
{
    double acc[kRedVals] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < kRedVals; ++k) acc[k] += partials[b * kRedVals + k];
    __shared__ double sm[kRedVals][kRedThreads];
#pragma unroll
    for (int k = 0; k < kRedVals; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kRedVals; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sm[0][0] + sm[1][0];   // sum rho = cells + sum h
        out[1] = sm[2][0];
        out[2] = sm[3][0];
        out[3] = sm[4][0];
        out[4] = sm[5][0];
    }
}

template <typename T>
__global__ void k_count_nonfinite(const T* f, const float* g, int64_t N, int64_t P,
                                  unsigned long long* count)
{
    unsigned long long bad = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int i = 0; i < Q; ++i) bad += !isfinite(Io<T>::ld(f + i * P + c));
        if (g)
#pragma unroll
            for (int i = 0; i < QS; ++i) bad += !isfinite(g[i * P + c]);
    }
    if (bad) atomicAdd(count, bad);
}

// ---------------------------------------------------------------------------
// host side: validation and launches
// ---------------------------------------------------------------------------
int64_t cells_of(const cslbm_level* L) { return (int64_t)L->nx * L->ny * L->nz; }

int validate_shape(const cslbm_level* L)
{
    if (!L) return fail(CSLBM_ERR_ARG, "level is NULL");
    if (L->nx < 1 || L->ny < 1 || L->nz < 1)
        return fail(CSLBM_ERR_SHAPE, "level size %d x %d x %d must be positive", L->nx, L->ny, L->nz);
    const int64_t N = cells_of(L);
    if (N > 0x7fffffffLL)
        return fail(CSLBM_ERR_SHAPE, "level has %lld cells; at most 2^31-1 are supported",
                    (long long)N);
    if (L->nz > 65535 || L->ny > 65535)
        return fail(CSLBM_ERR_SHAPE, "ny and nz must be at most 65535");
    if (L->plane < N)
        return fail(CSLBM_ERR_SHAPE, "plane stride %lld is smaller than nx*ny*nz = %lld",
                    (long long)L->plane, (long long)N);
    if (L->storage != CSLBM_F32 && L->storage != CSLBM_F16S)
        return fail(CSLBM_ERR_UNSUPPORTED, "unknown storage format %d", L->storage);
    if (!L->f) return fail(CSLBM_ERR_ARG, "f is NULL");
    if ((L->g == nullptr) != (L->g_next == nullptr))
        return fail(CSLBM_ERR_ARG, "g and g_next must both be set or both be NULL");
    if ((L->periodic & 7) != 7 && !L->flags)
        return fail(CSLBM_ERR_ARG, "a non-periodic axis needs a flags array (periodic = %d)",
                    L->periodic);
    return CSLBM_OK;
}

int validate_params(const cslbm_level* L)
{
    const cslbm_params& p = L->p;
    if (!(p.nu > 0.0) || !std::isfinite(p.nu))
        return fail(CSLBM_ERR_ARG, "viscosity nu = %g must be positive (S4..8 in (0, 2))", p.nu);
    for (int g = 0; g < 4; ++g)
        if (!(p.nu_hi[g] > 0.0) || !std::isfinite(p.nu_hi[g]))
            return fail(CSLBM_ERR_ARG, "artificial viscosity nu_hi[%d] = %g must be positive", g,
                        p.nu_hi[g]);
    if (p.adaptive) {
        if (!(p.g_max > 0.0)) return fail(CSLBM_ERR_ARG, "g_max = %g must be positive", p.g_max);
        if (!(p.b > 0.0) || !(p.a + p.b > 0.0))
            return fail(CSLBM_ERR_ARG,
                        "adaptive factor a*x + b must stay positive on [0, 1] (a = %g, b = %g)",
                        p.a, p.b);
    }
    if (L->g && !(p.tau_s > 0.5))
        return fail(CSLBM_ERR_ARG, "scalar relaxation time tau_s = %g must exceed 1/2", p.tau_s);
    if (p.grad_mode != 0 && p.grad_mode != 1)
        return fail(CSLBM_ERR_ARG, "grad_mode = %d must be 0 or 1", p.grad_mode);
    if (p.gmax_running && p.grad_mode != 1)
        return fail(CSLBM_ERR_ARG, "gmax_running needs grad_mode 1");
    return CSLBM_OK;
}

static inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// After the state of a gradient-mode level was written: its velocity field.
static int refresh_velocity(const cslbm_level* L, hipStream_t stream)
{
    if (L->p.grad_mode != 1 || !L->vel) return CSLBM_OK;
    const int64_t N = cells_of(L);
    const dim3 grid(blocks_for(N, 256)), block(256);
    const float beta = (float)L->p.beta, sref = (float)L->p.s_ref;
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_macro<float>, grid, block, 0, stream, (const float*)L->f, L->g, L->force,
                           N, L->plane, beta, sref, nullptr, L->vel, nullptr);
    else
        hipLaunchKernelGGL(k_macro<_Float16>, grid, block, 0, stream, (const _Float16*)L->f, L->g,
                           L->force, N, L->plane, beta, sref, nullptr, L->vel, nullptr);
    return check_launch("k_macro");
}

Rates make_rates(const cslbm_params& p)
{
    Rates r;
    r.S = (float)(1.0 / (3.0 * p.nu + 0.5));
    for (int g = 0; g < 4; ++g) r.nu3[g] = (float)(3.0 * p.nu_hi[g]);
    r.a = (float)p.a;
    r.b = (float)p.b;
    r.inv_gmax = p.adaptive ? (float)(1.0 / p.g_max) : 0.0f;
    r.adaptive = p.adaptive ? 1 : 0;
    return r;
}

// Block of 256 threads: bx consecutive x (a multiple of 64, so waves cover
// contiguous row segments) by 256/bx rows.  bx is the largest of 256, 128, 64
// that leaves the fewest idle lanes per row (nx = 384 -> 128, nx = 512 ->
// 256, nx = 96 -> 128).
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
                          float* gout);

// One step in the finite-difference gradient mode (grad_mode 1): the
// adaptive factor takes |grad u|_F of vel (the input state's velocity) and
// the new state's velocity goes to vel_out.
static int launch_step_grad(const cslbm_level* L, const void* fin, void* fout, const float* gin,
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
    return a;
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
    if (L->storage == CSLBM_F32)
        dispatch_step<float>(a, has_flags, has_force, has_scalar, time, stream);
    else
        dispatch_step<_Float16>(a, has_flags, has_force, has_scalar, time, stream);
    return check_launch("k_step");
}

}  // namespace cslbm

using namespace cslbm;

extern "C" {

int64_t cslbm_plane_stride(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(CSLBM_ERR_SHAPE, "sizes must be positive");
    const int64_t N = (int64_t)nx * ny * nz;
    // round up to 256 elements and add 3*256 so consecutive planes start at
    // offsets that differ by an odd number of 1 KiB blocks
    return ((N + 255) / 256) * 256 + 3 * 256;
}

int64_t cslbm_level_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t storage, int32_t with_scalar)
{
    const int64_t plane = cslbm_plane_stride(nx, ny, nz);
    if (plane < 0) return plane;
    if (storage != CSLBM_F32 && storage != CSLBM_F16S)
        return fail(CSLBM_ERR_UNSUPPORTED, "unknown storage format %d", storage);
    const int64_t elem = storage == CSLBM_F32 ? 4 : 2;
    return 27 * plane * elem + (with_scalar ? 7 * plane * 4 : 0);
}

int cslbm_prepare_flags(const cslbm_level* L, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!L->flags) return fail(CSLBM_ERR_ARG, "flags is NULL");
    const int64_t N = cells_of(L);
    hipLaunchKernelGGL(k_prepare_flags, dim3(blocks_for(N, 256)), dim3(256), 0, stream, L->flags,
                       L->links, L->nx, L->ny, L->nz, L->periodic);
    return check_launch("k_prepare_flags");
}

int cslbm_init_equilibrium(cslbm_level* L, const float* rho, const float* u, const float* s,
                           hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!u) return fail(CSLBM_ERR_ARG, "u is NULL");
    const int64_t N = cells_of(L);
    const dim3 grid(blocks_for(N, 256)), block(256);
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_init_eq<float>, grid, block, 0, stream, (float*)L->f, L->g, N, L->plane,
                           rho, u, s);
    else
        hipLaunchKernelGGL(k_init_eq<_Float16>, grid, block, 0, stream, (_Float16*)L->f, L->g, N,
                           L->plane, rho, u, s);
    rc = check_launch("k_init_eq");
    return rc ? rc : refresh_velocity(L, stream);
}

int cslbm_set_populations(cslbm_level* L, const float* f, const float* g, int32_t shifted,
                          hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!f) return fail(CSLBM_ERR_ARG, "source populations are NULL");
    const int64_t N = cells_of(L);
    const dim3 grid(blocks_for(N, 256)), block(256);
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_set_pop<float>, grid, block, 0, stream, (float*)L->f, L->g, N, L->plane,
                           f, g, shifted);
    else
        hipLaunchKernelGGL(k_set_pop<_Float16>, grid, block, 0, stream, (_Float16*)L->f, L->g, N,
                           L->plane, f, g, shifted);
    rc = check_launch("k_set_pop");
    return rc ? rc : refresh_velocity(L, stream);
}

int cslbm_get_populations(const cslbm_level* L, float* f, float* g, int32_t shifted,
                          hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!f) return fail(CSLBM_ERR_ARG, "destination is NULL");
    const int64_t N = cells_of(L);
    const dim3 grid(blocks_for(N, 256)), block(256);
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_get_pop<float>, grid, block, 0, stream, (const float*)L->f, L->g, N,
                           L->plane, f, g, shifted);
    else
        hipLaunchKernelGGL(k_get_pop<_Float16>, grid, block, 0, stream, (const _Float16*)L->f, L->g,
                           N, L->plane, f, g, shifted);
    return check_launch("k_get_pop");
}

int cslbm_copy_cells(const cslbm_level* src, const int32_t* src_cells, cslbm_level* dst,
                     const int32_t* dst_cells, int32_t n_cells, hipStream_t stream)
{
    int rc = validate_shape(src);
    if (rc) return rc;
    rc = validate_shape(dst);
    if (rc) return rc;
    if (src->storage != dst->storage)
        return fail(CSLBM_ERR_UNSUPPORTED, "copying between storage formats is not supported");
    if (n_cells < 0 || (n_cells > 0 && (!src_cells || !dst_cells)))
        return fail(CSLBM_ERR_ARG, "bad cell lists");
    if ((src->g != nullptr) != (dst->g != nullptr))
        return fail(CSLBM_ERR_ARG, "both levels or neither must carry the scalar");
    if (src->f == dst->f) return fail(CSLBM_ERR_ARG, "source and destination states alias");
    if (n_cells == 0) return CSLBM_OK;
    const dim3 grid(blocks_for(n_cells, 256)), block(256);
    if (src->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_copy_cells<float>, grid, block, 0, stream, (const float*)src->f, src->g,
                           src->plane, (float*)dst->f, dst->g, dst->plane, src_cells, dst_cells,
                           n_cells);
    else
        hipLaunchKernelGGL(k_copy_cells<_Float16>, grid, block, 0, stream, (const _Float16*)src->f,
                           src->g, src->plane, (_Float16*)dst->f, dst->g, dst->plane, src_cells,
                           dst_cells, n_cells);
    return check_launch("k_copy_cells");
}

int cslbm_step(cslbm_level* L, int32_t n_steps, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    rc = validate_params(L);
    if (rc) return rc;
    if (n_steps < 0) return fail(CSLBM_ERR_ARG, "n_steps = %d is negative", n_steps);
    if (!L->f_next) return fail(CSLBM_ERR_ARG, "f_next is NULL");
    if (L->f == L->f_next) return fail(CSLBM_ERR_ARG, "f and f_next alias");
    if (L->g && L->g == L->g_next) return fail(CSLBM_ERR_ARG, "g and g_next alias");
    const bool grad = L->p.grad_mode == 1;
    if (grad) {
        if (L->flags)
            return fail(CSLBM_ERR_UNSUPPORTED,
                        "the finite-difference gradient mode needs a fully periodic level without flags");
        if (!L->vel || !L->vel_next || L->vel == L->vel_next)
            return fail(CSLBM_ERR_ARG, "grad_mode 1 needs distinct vel and vel_next buffers");
        if (L->p.gmax_running && !L->gmax_buf)
            return fail(CSLBM_ERR_ARG, "gmax_running needs gmax_buf");
    }

    for (int n = 0; n < n_steps; ++n) {
        rc = grad ? launch_step_grad(L, L->f, L->f_next, L->g, L->g_next, L->vel, L->vel_next, stream)
                  : launch_step_into(L, L->f, L->f_next, L->g, L->g_next, stream);
        if (rc) return rc;
        if (grad) std::swap(L->vel, L->vel_next);
        void* t = L->f;
        L->f = L->f_next;
        L->f_next = t;
        float* tg = L->g;
        L->g = L->g_next;
        L->g_next = tg;
    }
    return CSLBM_OK;
}

int cslbm_read_macro(const cslbm_level* L, float* rho, float* u, float* s, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (s && !L->g) return fail(CSLBM_ERR_ARG, "scalar requested but the level has no g");
    const int64_t N = cells_of(L);
    const dim3 grid(blocks_for(N, 256)), block(256);
    const float beta = (float)L->p.beta, sref = (float)L->p.s_ref;
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_macro<float>, grid, block, 0, stream, (const float*)L->f, L->g, L->force,
                           N, L->plane, beta, sref, rho, u, s);
    else
        hipLaunchKernelGGL(k_macro<_Float16>, grid, block, 0, stream, (const _Float16*)L->f, L->g,
                           L->force, N, L->plane, beta, sref, rho, u, s);
    return check_launch("k_macro");
}

int cslbm_vorticity(const cslbm_level* L, float* omega, float* speed, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!omega) return fail(CSLBM_ERR_ARG, "omega is NULL");
    const int64_t N = cells_of(L);
    float* u = nullptr;
    CSLBM_HIP_TRY(hipMallocAsync((void**)&u, 3 * N * sizeof(float), stream));
    const dim3 grid(blocks_for(N, 256)), block(256);
    const float beta = (float)L->p.beta, sref = (float)L->p.s_ref;
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_macro<float>, grid, block, 0, stream, (const float*)L->f, L->g, L->force,
                           N, L->plane, beta, sref, nullptr, u, nullptr);
    else
        hipLaunchKernelGGL(k_macro<_Float16>, grid, block, 0, stream, (const _Float16*)L->f, L->g,
                           L->force, N, L->plane, beta, sref, nullptr, u, nullptr);
    rc = check_launch("k_macro");
    if (!rc) {
        hipLaunchKernelGGL(k_vorticity, grid, block, 0, stream, u, L->nx, L->ny, L->nz,
                           L->periodic & 7, omega, speed);
        rc = check_launch("k_vorticity");
    }
    const hipError_t ef = hipFreeAsync(u, stream);
    if (rc) return rc;
    if (ef != hipSuccess) return fail(CSLBM_ERR_HIP, "hipFreeAsync: %s", hipGetErrorString(ef));
    return CSLBM_OK;
}

int cslbm_conserved_f64(const cslbm_level* L, double out[5], hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!out) return fail(CSLBM_ERR_ARG, "out is NULL");
    const int64_t N = cells_of(L);
    double* dmem = nullptr;
    CSLBM_HIP_TRY(hipMallocAsync((void**)&dmem, (kRedBlocks * kRedVals + 8) * sizeof(double), stream));
    double* partials = dmem;
    double* dout = dmem + kRedBlocks * kRedVals;
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_conserved_partials<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                           (const float*)L->f, L->g, L->flags, N, L->plane, partials);
    else
        hipLaunchKernelGGL(k_conserved_partials<_Float16>, dim3(kRedBlocks), dim3(kRedThreads), 0,
                           stream, (const _Float16*)L->f, L->g, L->flags, N, L->plane, partials);
    rc = check_launch("k_conserved_partials");
    if (!rc) {
        hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(kRedThreads), 0, stream, partials,
                           kRedBlocks, dout);
        rc = check_launch("k_conserved_final");
    }
    double host[5] = {0, 0, 0, 0, 0};
    if (!rc) {
        const hipError_t e = hipMemcpyAsync(host, dout, sizeof host, hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) rc = fail(CSLBM_ERR_HIP, "copy of the totals: %s", hipGetErrorString(e));
    }
    const hipError_t ef = hipFreeAsync(dmem, stream);
    const hipError_t es = hipStreamSynchronize(stream);
    if (rc) return rc;
    if (ef != hipSuccess) return fail(CSLBM_ERR_HIP, "hipFreeAsync: %s", hipGetErrorString(ef));
    if (es != hipSuccess) return fail(CSLBM_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
    std::memcpy(out, host, sizeof host);
    return CSLBM_OK;
}

int cslbm_check_finite(const cslbm_level* L, int64_t* n_bad, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!n_bad) return fail(CSLBM_ERR_ARG, "n_bad is NULL");
    const int64_t N = cells_of(L);
    unsigned long long* dcount = nullptr;
    CSLBM_HIP_TRY(hipMallocAsync((void**)&dcount, sizeof(unsigned long long), stream));
    rc = CSLBM_OK;
    hipError_t e = hipMemsetAsync(dcount, 0, sizeof(unsigned long long), stream);
    if (e != hipSuccess) rc = fail(CSLBM_ERR_HIP, "hipMemsetAsync: %s", hipGetErrorString(e));
    if (!rc) {
        const unsigned nb = (unsigned)std::min<int64_t>(blocks_for(N, 256), 4096);
        if (L->storage == CSLBM_F32)
            hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(nb), dim3(256), 0, stream,
                               (const float*)L->f, L->g, N, L->plane, dcount);
        else
            hipLaunchKernelGGL(k_count_nonfinite<_Float16>, dim3(nb), dim3(256), 0, stream,
                               (const _Float16*)L->f, L->g, N, L->plane, dcount);
        rc = check_launch("k_count_nonfinite");
    }
    unsigned long long host = 0;
    if (!rc) {
        e = hipMemcpyAsync(&host, dcount, sizeof host, hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) rc = fail(CSLBM_ERR_HIP, "copy of the count: %s", hipGetErrorString(e));
    }
    const hipError_t ef = hipFreeAsync(dcount, stream);
    const hipError_t es = hipStreamSynchronize(stream);
    if (rc) return rc;
    if (ef != hipSuccess) return fail(CSLBM_ERR_HIP, "hipFreeAsync: %s", hipGetErrorString(ef));
    if (es != hipSuccess) return fail(CSLBM_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(es));
    *n_bad = (int64_t)host;
    if (host) return fail(CSLBM_ERR_NONFINITE, "%llu non-finite values in the state", host);
    return CSLBM_OK;
}

int cslbm_abi_sizes(int64_t* params_bytes, int64_t* level_bytes)
{
    if (params_bytes) *params_bytes = (int64_t)sizeof(cslbm_params);
    if (level_bytes) *level_bytes = (int64_t)sizeof(cslbm_level);
    return CSLBM_OK;
}

const char* cslbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
