// lattice.hpp -- D3Q27 / D3Q7 lattice constants for the GPU path (gfx950).
//
// Population index i follows the velocity list of the paper's appendix
// (entry 13 of c_z taken as -1, which makes the 27 velocities the full cube
// {-1,0,1}^3).  Inside a kernel the 27 values of a cell live in registers in
// "tensor order" t = (cx+1) + 3(cy+1) + 9(cz+1), so that the central-moment
// transform factorises into sweeps along x, y and z.  After the forward sweeps
// slot t holds the raw central moment k_mnp with (m, n, p) the same digits.
#pragma once

#include <cstdint>

namespace cslbm {

constexpr int Q = 27;
constexpr int QS = 7;

// appendix velocity list, paper order
constexpr int kCx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                        0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int kCy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1,
                        -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int kCz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1,
                        1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

// tensor slot of paper index i
constexpr int tensor_slot(int i) { return (kCx[i] + 1) + 3 * (kCy[i] + 1) + 9 * (kCz[i] + 1); }

// lattice weight: product of the 1D weights 2/3 (c = 0), 1/6 (c = +-1)
constexpr float weight1d(int c) { return c == 0 ? 2.0f / 3.0f : 1.0f / 6.0f; }
constexpr float weight(int i) { return weight1d(kCx[i]) * weight1d(kCy[i]) * weight1d(kCz[i]); }

constexpr int opposite(int i)
{
    for (int k = 0; k < Q; ++k)
        if (kCx[k] == -kCx[i] && kCy[k] == -kCy[i] && kCz[k] == -kCz[i]) return k;
    return -1;
}

// D3Q7 passive-scalar lattice: rest, +x, -x, +y, -y, +z, -z
constexpr int kSx[QS] = {0, 1, -1, 0, 0, 0, 0};
constexpr int kSy[QS] = {0, 0, 0, 1, -1, 0, 0};
constexpr int kSz[QS] = {0, 0, 0, 0, 0, 1, -1};
constexpr float kSw[QS] = {0.25f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f};
constexpr int scalar_opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// tensor slot of the moment k_mnp
constexpr int kslot(int m, int n, int p) { return m + 3 * n + 9 * p; }

// cell kinds (low 3 bits of the flag byte)
enum : uint8_t {
    kFluid = 0,
    kSolid = 1,
    kInlet = 2,
    kOutflow = 3,
    kGhost = 4,
    kNeumann = 5,
    kWall = 6,
};
constexpr uint8_t kKindMask = 0x07;
constexpr uint8_t kNearWall = 0x08;  // set by the library: some pull source is solid
constexpr int kWallNormalShift = 5;  // wall cells: normal code 1..6 (7: not a flat wall)

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


static_assert(tensor_slot(0) == 13, "rest velocity sits in the middle of the cube");
static_assert(tensor_slot(13) == 2 + 3 * 1 + 9 * 0, "erratum: velocity 13 is (1,0,-1)");

}  // namespace cslbm
