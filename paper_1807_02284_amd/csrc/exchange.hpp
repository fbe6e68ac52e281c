// exchange.hpp -- arguments and stencil geometry of the cross-scale
// exchange (section "Spatial scale mapping"), shared by the exchange kernels
// and their adjoints.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/cslbm.h"
#include "brick.hpp"

namespace cslbm {

struct ExchArgs {
    const void* fA;
    const void* fB;
    const float* gA;
    const float* gB;
    int snx, sny, snz, speriodic;
    int64_t splane;
    double sorigin[3], sdx;
    void* fo;
    float* go;
    int dnx, dny, dnz;
    BrickMap sb, db;      // brick storage of source and destination (table null: dense)
    int64_t dplane;
    double dorigin[3], ddx;
    const int32_t* cells;
    int n_cells;
    float w;
    float kappa;     // stress rescaling
    float kappa_s;   // scalar non-equilibrium rescaling
    // Staged segments (forward exchange only): the first list entries are
    // mapped from compact copies of sub-boxes of the source level instead
    // of the source level itself.  Segment s covers list entries
    // [st[s].first, st[s].first + st[s].count) and the first st[s].blocks
    // blocks after the previous segments; the remaining blocks map entries
    // [main_first, n_cells) from the source level.  A staged copy starts at
    // source cell st[s].off: the stencil geometry is still that of the source
    // level (same weights and corners), only the corner indices are shifted.
    // A corner outside the copy (a list entry that does not belong to its
    // face) makes the target NaN instead of reading a clamped cell.
    struct Staged {
        const void* fA;
        const void* fB;
        const float* gA;
        const float* gB;
        int nx, ny, nz;
        int off[3];
        int64_t plane;
        int first, count, blocks;
    };
    int n_staged;
    int main_first;
    Staged st[2];
};

// The workgroups of a launch are handed out to the 8 XCDs in turn (hardware
// block b, in dispatch order, runs on XCD b % 8), and each XCD has its own
// L2.  xcd_block maps the hardware block index to a logical one so that
// every XCD walks one contiguous range of logical blocks: blocks that share
// cache lines meet in the same L2.  A bijection of [0, nb): XCD x runs
// nb / 8 blocks, one more if x < nb % 8.
__host__ __device__ constexpr int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

constexpr bool xcd_block_is_bijective(int nb)
{
    bool seen[64] = {};
    for (int b = 0; b < nb; ++b) {
        const int l = xcd_block(b, nb);
        if (l < 0 || l >= nb || seen[l]) return false;
        seen[l] = true;
    }
    return true;
}
static_assert(xcd_block_is_bijective(1) && xcd_block_is_bijective(7) && xcd_block_is_bijective(8) &&
                  xcd_block_is_bijective(13) && xcd_block_is_bijective(64),
              "xcd_block must permute the blocks");

__device__ __forceinline__ int wrap_or_clamp(int i, int n, bool periodic)
{
    if (periodic) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);   // lists are validated on the host
}

// target point of list entry k in source lattice coordinates: base corner
// and trilinear fractions (geometry in FP64 so coincident nodes resolve)
__device__ __forceinline__ void target_stencil(const ExchArgs& a, int c, int (&base)[3], float (&t)[3])
{
    int x, y, z;
    if (a.db.table) {
        brick_xyz(a.db, c, x, y, z);
    } else {
        x = c % a.dnx;
        y = (c / a.dnx) % a.dny;
        z = c / (a.dnx * a.dny);
    }
    const double p[3] = {a.dorigin[0] + x * a.ddx, a.dorigin[1] + y * a.ddx, a.dorigin[2] + z * a.ddx};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double q = (p[d] - a.sorigin[d]) / a.sdx;
        const double b = floor(q);
        base[d] = (int)b;
        t[d] = (float)(q - b);
    }
}

// storage index of source corner (ix, iy, iz) (inside the source box); a
// corner in a brick that is not stored reads cell 0 (validated lists never
// put weight on one)
__device__ __forceinline__ int64_t source_cell(const ExchArgs& a, int ix, int iy, int iz)
{
    if (a.sb.table) {
        const int s = brick_cell(a.sb, ix, iy, iz);
        return s < 0 ? 0 : s;
    }
    return ix + (int64_t)a.snx * (iy + (int64_t)a.sny * iz);
}

__device__ __forceinline__ float corner_weight(const float (&t)[3], int corner)
{
    const int ox = corner & 1, oy = (corner >> 1) & 1, oz = (corner >> 2) & 1;
    return (ox ? t[0] : 1.0f - t[0]) * (oy ? t[1] : 1.0f - t[1]) * (oz ? t[2] : 1.0f - t[2]);
}

inline double shear_rate(const cslbm_level* L) { return 1.0 / (3.0 * L->p.nu + 0.5); }

// Every target lies on a source lattice point: the target spacing is a whole
// multiple of the source spacing and the origins are whole source cells apart.
inline bool nodes_coincide(const cslbm_level* src, const cslbm_level* dst)
{
    const double r = dst->dx / src->dx;
    if (!(r >= 1.0 - 1e-9) || std::fabs(r - std::nearbyint(r)) > 1e-9) return false;
    for (int d = 0; d < 3; ++d) {
        const double o = (dst->origin[d] - src->origin[d]) / src->dx;
        if (std::fabs(o - std::nearbyint(o)) > 1e-9) return false;
    }
    return true;
}

// Kernel arguments of one exchange from src (states fA, fB blended with
// weight w) to the listed cells of dst (outputs f_out, g_out).
inline ExchArgs exchange_args(const cslbm_level* src, const void* fA, const void* fB,
                              const float* gA, const float* gB, double w, const cslbm_level* dst,
                              void* f_out, float* g_out, const int32_t* cells, int32_t n_cells)
{
    ExchArgs a;
    a.fA = fA;
    a.fB = fB ? fB : fA;
    const bool scalar = gA && g_out;
    a.gA = scalar ? gA : nullptr;
    a.gB = scalar ? (gB ? gB : gA) : nullptr;
    a.snx = src->nx;
    a.sny = src->ny;
    a.snz = src->nz;
    a.speriodic = src->periodic & 7;
    a.splane = src->plane;
    std::memcpy(a.sorigin, src->origin, sizeof a.sorigin);
    a.sdx = src->dx;
    a.fo = f_out;
    a.go = scalar ? g_out : nullptr;
    a.dnx = dst->nx;
    a.dny = dst->ny;
    a.dnz = dst->nz;
    a.dplane = dst->plane;
    std::memcpy(a.dorigin, dst->origin, sizeof a.dorigin);
    a.ddx = dst->dx;
    a.sb = brick_map(src);
    a.db = brick_map(dst);
    a.cells = cells;
    a.n_cells = n_cells;
    a.w = (float)w;
    a.n_staged = 0;
    a.main_first = 0;
    const double alpha = src->dx / dst->dx;
    const double Ss = shear_rate(src), Sd = shear_rate(dst);
    a.kappa = (float)((1.0 - Sd) / (1.0 - Ss) * Ss / (alpha * Sd));
    a.kappa_s = scalar ? (float)((dst->p.tau_s - 1.0) / (alpha * (src->p.tau_s - 1.0))) : 0.0f;
    return a;
}

// One exchange launch (validated arguments); defined with the kernels.
// With runs (n_runs + 1 offsets grouping the list into runs of at most 256
// entries), an exchange from a dense source into a dense destination that
// the tiled kernel handles maps one run per workgroup through LDS.
int launch_exchange(const cslbm_level* src, const void* fA, const void* fB, const float* gA,
                    const float* gB, double w, const cslbm_level* dst, void* f_out, float* g_out,
                    const int32_t* cells, int32_t n_cells, hipStream_t stream,
                    const int32_t* runs = nullptr, int32_t n_runs = 0);

// Prior-mapping of finer scale sc's boundary shell from its parent P
// (states A at t_n and B at t_n + dt_0, time weight w).  prior_stage copies
// the parent's columns around the shell's two planes normal to x into
// sc.stage when the scale has them listed and a stage (sets *staged);
// prior_map then reads those planes' stencils from the copy, bitwise the
// same result as reading the parent.  Arguments validated.
int prior_stage(const cslbm_scale& sc, const cslbm_level* P, const void* A, const void* B,
                const float* gA, const float* gB, bool* staged, hipStream_t stream);
int prior_map(const cslbm_scale& sc, bool staged, const cslbm_level* P, const void* A, const void* B,
              const float* gA, const float* gB, double w, void* out, float* gout, hipStream_t stream);
// The staged segments of that prior-mapping (a built by exchange_args over
// sc's ghost list): false, a unchanged, when it is not staged.
bool prior_segments(const cslbm_scale& sc, bool staged, const cslbm_level* P, ExchArgs& a);

// Adjoint of one collide-stream step of level L from the input state
// (fin, gin): lam = dL/d(input) from lam_next = dL/d(output) (likewise mu for
// the scalar), dtheta accumulated when not null.  Arguments validated.
int launch_adjoint_into(const cslbm_level* L, const void* fin, const float* gin,
                        const float* lam_next, const float* mu_next, float* lam, float* mu,
                        float* dtheta, hipStream_t stream);

// Checks of a hierarchy (scale kinds, parents, lists, buffers) shared by the
// multi-scale step and its adjoint; 0 or an error code with the message set.
int validate_hierarchy(const cslbm_hierarchy* H);

}  // namespace cslbm
