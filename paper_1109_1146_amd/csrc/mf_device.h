// Shared device-side definitions of the region-discharge solver (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfd {

constexpr int kMaxK = 8;
constexpr int32_t kInf = 0x7fffffff;
constexpr int kHistBins = 1 << 16;  // boundary-label histogram bins (labels beyond are not gap candidates)
constexpr int kHistLds = 1024;      // per-block privatised histogram bins

// The canonical 2D directions k = 0..7 as (dy, dx): +x, -x, +y, -y, then the
// diagonals (+y+x), (-y-x), (-y+x), (+y-x); the reverse of direction k is k ^ 1
// and 4-connected grids use k < 4.  Kernels that only run on 2D grids take the
// offsets from here, so that they are compile-time constants.
__host__ __device__ constexpr int off2d_dy(int k) {
    return (k == 2 || k == 4 || k == 7) ? 1 : ((k == 3 || k == 5 || k == 6) ? -1 : 0);
}
__host__ __device__ constexpr int off2d_dx(int k) {
    return (k == 0 || k == 4 || k == 6) ? 1 : ((k == 1 || k == 5 || k == 7) ? -1 : 0);
}

// Grid geometry in blocked (region-major) layout.  2D grids are stored as
// depth-1 3D grids.  A region is a tz x ty x tx box; its V vertices are
// contiguous, x fastest; regions are numbered z-major over the region grid.
struct Geo {
    int K;
    int dz, dy, dx;   // real grid extents
    int tz, ty, tx;   // region (tile) extents
    int rz, ry, rx;   // number of regions per axis
    int V;            // tz * ty * tx
    int nreg;
    int N;            // nreg * V (padded vertex count, < 2^31)
    int8_t oz[kMaxK], oy[kMaxK], ox[kMaxK];
};

__device__ __forceinline__ void local_xyz(const Geo &G, int l, int &z, int &y, int &x) {
    x = l % G.tx;
    int t = l / G.tx;
    y = t % G.ty;
    z = t / G.ty;
}

__device__ __forceinline__ void region_xyz(const Geo &G, int r, int &z, int &y, int &x) {
    x = r % G.rx;
    int t = r / G.rx;
    y = t % G.ry;
    z = t / G.ry;
}

// Local index of the in-tile neighbour in direction k, or -1 if the arc leaves the tile.
__device__ __forceinline__ int local_nbr(const Geo &G, int lz, int ly, int lx, int k) {
    int z = lz + G.oz[k], y = ly + G.oy[k], x = lx + G.ox[k];
    if ((unsigned)x >= (unsigned)G.tx || (unsigned)y >= (unsigned)G.ty || (unsigned)z >= (unsigned)G.tz)
        return -1;
    return (z * G.ty + y) * G.tx + x;
}

// Blocked index of the neighbour across the tile border in direction k, or -1
// when it falls outside the region grid.  Only valid when local_nbr() == -1.
__device__ __forceinline__ int cross_nbr(const Geo &G, int r, int lz, int ly, int lx, int k) {
    int z = lz + G.oz[k], y = ly + G.oy[k], x = lx + G.ox[k];
    int rz, ry, rx;
    region_xyz(G, r, rz, ry, rx);
    if (x < 0) { x += G.tx; rx--; } else if (x >= G.tx) { x -= G.tx; rx++; }
    if (y < 0) { y += G.ty; ry--; } else if (y >= G.ty) { y -= G.ty; ry++; }
    if (z < 0) { z += G.tz; rz--; } else if (z >= G.tz) { z -= G.tz; rz++; }
    if ((unsigned)rx >= (unsigned)G.rx || (unsigned)ry >= (unsigned)G.ry || (unsigned)rz >= (unsigned)G.rz)
        return -1;
    return ((rz * G.ry + ry) * G.rx + rx) * G.V + (z * G.ty + y) * G.tx + x;
}

// Blocked index -> real grid coordinates; returns false for padding vertices.
__device__ __forceinline__ bool blocked_to_grid(const Geo &G, int g, int &z, int &y, int &x) {
    int r = g / G.V, l = g - r * G.V;
    int lz, ly, lx, rz, ry, rx;
    local_xyz(G, l, lz, ly, lx);
    region_xyz(G, r, rz, ry, rx);
    z = rz * G.tz + lz;
    y = ry * G.ty + ly;
    x = rx * G.tx + lx;
    return z < G.dz && y < G.dy && x < G.dx;
}

__device__ __forceinline__ int grid_to_blocked(const Geo &G, int z, int y, int x) {
    int rz = z / G.tz, ry = y / G.ty, rx = x / G.tx;
    int lz = z - rz * G.tz, ly = y - ry * G.ty, lx = x - rx * G.tx;
    return ((rz * G.ry + ry) * G.rx + rx) * G.V + (lz * G.ty + ly) * G.tx + lx;
}

}  // namespace mfd
