// brick.hpp -- sparse brick storage of a level (build addition for thin
// dynamic regions): the level's box is tiled by 8x8x8 bricks and only the
// active bricks are stored, one after another, each as 512 cells in x-fastest
// order (storage index = 512 * brick + lx + 8 ly + 64 lz).  A dense table
// over the brick grid gives each brick's index (-1: not stored) and each
// stored brick's coordinates are kept for the inverse map.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/cslbm.h"

namespace cslbm {

constexpr int kBrickEdge = 8;
constexpr int kBrickCells = 512;

struct BrickMap {
    const int32_t* table;    // [bnz][bny][bnx] brick index or -1; null: dense box
    const int32_t* origin;   // [n_bricks][3] brick coordinates
    int bnx, bny, bnz;
};

// storage index of box cell (x, y, z); -1 outside the box or in a brick
// that is not stored
__host__ __device__ __forceinline__ int brick_cell(const BrickMap& m, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0) return -1;
    const int bx = x >> 3, by = y >> 3, bz = z >> 3;
    if (bx >= m.bnx || by >= m.bny || bz >= m.bnz) return -1;
    const int b = m.table[bx + m.bnx * (by + m.bny * bz)];
    return b < 0 ? -1 : (b << 9) + (x & 7) + ((y & 7) << 3) + ((z & 7) << 6);
}

// box coordinates of storage index c
__host__ __device__ __forceinline__ void brick_xyz(const BrickMap& m, int c, int& x, int& y, int& z)
{
    const int b = c >> 9, l = c & 511;
    x = (m.origin[3 * b] << 3) + (l & 7);
    y = (m.origin[3 * b + 1] << 3) + ((l >> 3) & 7);
    z = (m.origin[3 * b + 2] << 3) + (l >> 6);
}

// storage index of box cell (x - cx, y - cy, z - cz) seen from storage index
// c at (x, y, z): an offset inside the brick, else through the table; -1 if
// that cell is not stored
__host__ __device__ __forceinline__ int brick_neighbour(const BrickMap& m, int c, int x, int y, int z,
                                                        int cx, int cy, int cz)
{
    const int lx = (x & 7) - cx, ly = (y & 7) - cy, lz = (z & 7) - cz;
    if ((unsigned)lx < 8u && (unsigned)ly < 8u && (unsigned)lz < 8u)
        return c - cx - (cy << 3) - (cz << 6);
    return brick_cell(m, x - cx, y - cy, z - cz);
}

// Brick map of a level (table null for a dense box).
BrickMap brick_map(const cslbm_level* L);

}  // namespace cslbm
