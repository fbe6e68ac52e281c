// cslbm.hip -- the C ABI of libcslbm (gfx950) and its single-level helper
// kernels: flags, initialisation, population copies, read-back, vorticity,
// FP64 conservation totals and the finiteness check.  The collide-stream
// kernel itself lives in step.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "../../include/cslbm.h"
#include "cm_collide.hpp"
#include "brick.hpp"
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
// auxiliary kernels (one thread per cell, 1D launch over N)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cell_coords(int64_t c, int nx, int ny, int& x, int& y, int& z)
{
    x = (int)(c % nx);
    y = (int)((c / nx) % ny);
    z = (int)(c / ((int64_t)nx * ny));
}

__global__ void k_prepare_flags(uint8_t* flags, uint32_t* links, int nx, int ny, int nz,
                                int periodic, int64_t N, const BrickMap bm)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    int x, y, z;
    if (bm.table)
        brick_xyz(bm, (int)c, x, y, z);
    else
        cell_coords(c, nx, ny, x, y, z);
    const uint8_t kind = flags[c] & kKindMask;
    uint32_t m = 0;
    bool near_fluid = false;
    if (kind != kFluid && kind != kWall) {
        // some neighbour (periodic wrap on every axis) is fluid: the adjoint
        // step checks such cells' neighbours before writing zeros
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            int64_t src;
            if (bm.table) {
                const int s = brick_neighbour(bm, (int)c, x, y, z, kCx[i], kCy[i], kCz[i]);
                if (s < 0) continue;
                src = s;
            } else {
                const int xs = (x - kCx[i] + nx) % nx, ys = (y - kCy[i] + ny) % ny,
                          zs = (z - kCz[i] + nz) % nz;
                src = xs + (int64_t)nx * (ys + (int64_t)ny * zs);
            }
            near_fluid |= (flags[src] & kKindMask) == kFluid;
        }
    } else {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (leaves_box(x, y, z, kCx[i], kCy[i], kCz[i], nx, ny, nz, periodic)) {
                m |= 1u << i;
                continue;
            }
            int64_t src;
            if (bm.table) {
                // a source that is not stored counts as solid (a valid brick
                // level never lets a fluid cell pull from one)
                const int s = brick_neighbour(bm, (int)c, x, y, z, kCx[i], kCy[i], kCz[i]);
                if (s < 0) {
                    m |= 1u << i;
                    continue;
                }
                src = s;
            } else {
                const int xs = (x - kCx[i] + nx) % nx, ys = (y - kCy[i] + ny) % ny,
                          zs = (z - kCz[i] + nz) % nz;
                src = xs + (int64_t)nx * (ys + (int64_t)ny * zs);
            }
            if ((flags[src] & kKindMask) == kSolid) m |= 1u << i;
        }
    }
    // wall node: the normal is minus the one axis velocity whose pull source
    // is blocked (code k for velocity k = 1..6: n = -c_k), and the blocked
    // sources must be exactly those of the velocities pointing away from the
    // wall (c.n < 0); otherwise code 7
    int wall_code = 0;
    if (kind == kWall) {
        int axis_blocked = 0;
        wall_code = 7;
#pragma unroll
        for (int k = 1; k <= 6; ++k)
            if (m & (1u << k)) {
                ++axis_blocked;
                wall_code = k;
            }
        if (axis_blocked != 1) {
            wall_code = 7;
        } else {
            uint32_t expect = 0;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int cn = -(kCx[i] * kCx[wall_code] + kCy[i] * kCy[wall_code] +
                                 kCz[i] * kCz[wall_code]);
                if (cn < 0) expect |= 1u << i;
            }
            if (expect != m) wall_code = 7;
        }
    }
    flags[c] = kind | (m ? kNearWall : 0) | (near_fluid ? CSLBM_NEAR_FLUID : 0) |
               (uint8_t)(wall_code << kWallNormalShift);
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
    float v[Q], u[QS];   // all loads before the first store
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = src[i * N + c];
    const bool scalar = g && gsrc;
    if (scalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) u[i] = gsrc[i * N + c];
#pragma unroll
    for (int i = 0; i < Q; ++i) Io<T>::st(f + i * P + c, shifted ? v[i] : v[i] - weight(i));
    if (scalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) g[i * P + c] = u[i];
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
    // all loads before the first store: a store between them would order
    // each later load after it (the compiler cannot rule out overlap)
    T v[Q];
    float u[QS];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = f[i * P + a];
    if (g)
#pragma unroll
        for (int i = 0; i < QS; ++i) u[i] = g[i * P + a];
#pragma unroll
    for (int i = 0; i < Q; ++i) fo[i * Po + b] = v[i];
    if (g)
#pragma unroll
        for (int i = 0; i < QS; ++i) go[i * Po + b] = u[i];
}

template <typename T>
__global__ void k_get_pop(const T* f, const float* g, int64_t N, int64_t P, float* dst, float* gdst,
                          int shifted)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    float h[Q], u[QS];   // all loads before the first store
#pragma unroll
    for (int i = 0; i < Q; ++i) h[i] = Io<T>::ld(f + i * P + c);
    const bool scalar = g && gdst;
    if (scalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) u[i] = g[i * P + c];
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[i * N + c] = shifted ? h[i] : h[i] + weight(i);
    if (scalar)
#pragma unroll
        for (int i = 0; i < QS; ++i) gdst[i * N + c] = u[i];
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

// Scratch of the allocation-free conservation call: the per-block partials
// of k_conserved_partials (every block writes its own entries, so nothing
// needs clearing between calls).  One copy per GPU, held until the process
// ends; host code uses the device address from hipGetSymbolAddress, never
// the symbol itself.
constexpr int64_t kScratchDoubles = (int64_t)kRedBlocks * kRedVals;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
static int scratch_of_current_device(double** out)
{
    int dev = -1;
    CSLBM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(CSLBM_ERR_UNSUPPORTED, "device index %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(CSLBM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return CSLBM_OK;
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
int64_t cells_of(const cslbm_level* L)
{
    return L->brick_table ? (int64_t)L->n_bricks * kBrickCells : (int64_t)L->nx * L->ny * L->nz;
}

BrickMap brick_map(const cslbm_level* L)
{
    BrickMap m;
    m.table = L->brick_table;
    m.origin = L->brick_origin;
    m.bnx = L->nx / kBrickEdge;
    m.bny = L->ny / kBrickEdge;
    m.bnz = L->nz / kBrickEdge;
    return m;
}

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
    if (L->wall_cells < 0 || (L->wall_cells > 0 && !L->flags))
        return fail(CSLBM_ERR_ARG, "wall_cells = %d needs a flags array holding them", L->wall_cells);
    if (L->brick_table) {
        if (L->nx % kBrickEdge || L->ny % kBrickEdge || L->nz % kBrickEdge)
            return fail(CSLBM_ERR_SHAPE, "a brick level's box %d x %d x %d must be a multiple of 8",
                        L->nx, L->ny, L->nz);
        const int64_t nb = (int64_t)(L->nx / 8) * (L->ny / 8) * (L->nz / 8);
        if (L->n_bricks < 1 || L->n_bricks > nb)
            return fail(CSLBM_ERR_ARG, "n_bricks = %d outside [1, %lld]", L->n_bricks, (long long)nb);
        if (!L->brick_origin) return fail(CSLBM_ERR_ARG, "brick_origin is NULL");
        if (!L->flags) return fail(CSLBM_ERR_ARG, "a brick level needs flags");
        if (L->periodic & 7) return fail(CSLBM_ERR_UNSUPPORTED, "a brick level has no periodic axis");
        if (L->force) return fail(CSLBM_ERR_UNSUPPORTED, "a brick level has no force field");
    }
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
                       L->links, L->nx, L->ny, L->nz, L->periodic, N, brick_map(L));
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
    if (L->brick_table) return fail(CSLBM_ERR_UNSUPPORTED, "vorticity of a brick level");
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

int cslbm_conserved_f64_noalloc(const cslbm_level* L, double* totals, hipStream_t stream)
{
    int rc = validate_shape(L);
    if (rc) return rc;
    if (!totals) return fail(CSLBM_ERR_ARG, "totals is NULL");
    // the reduction grid is fixed (grid-stride loop), so every level fits
    static_assert((int64_t)kRedBlocks * kRedVals <= kScratchDoubles, "partials exceed the scratch");
    double* partials = nullptr;
    rc = scratch_of_current_device(&partials);
    if (rc) return rc;
    const int64_t N = cells_of(L);
    if (L->storage == CSLBM_F32)
        hipLaunchKernelGGL(k_conserved_partials<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                           (const float*)L->f, L->g, L->flags, N, L->plane, partials);
    else
        hipLaunchKernelGGL(k_conserved_partials<_Float16>, dim3(kRedBlocks), dim3(kRedThreads), 0,
                           stream, (const _Float16*)L->f, L->g, L->flags, N, L->plane, partials);
    rc = check_launch("k_conserved_partials");
    if (rc) return rc;
    hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(kRedThreads), 0, stream, partials,
                       kRedBlocks, totals);
    return check_launch("k_conserved_final");
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

int cslbm_abi_sizes(int64_t* params_bytes, int64_t* level_bytes, int64_t* scale_bytes)
{
    if (params_bytes) *params_bytes = (int64_t)sizeof(cslbm_params);
    if (level_bytes) *level_bytes = (int64_t)sizeof(cslbm_level);
    if (scale_bytes) *scale_bytes = (int64_t)sizeof(cslbm_scale);
    return CSLBM_OK;
}

const char* cslbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
