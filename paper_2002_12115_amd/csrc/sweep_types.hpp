// sweep_types.hpp -- data types shared by the sweep kernels and the runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace hj {

constexpr int kWave = 64;

// Coefficient slots inside Grid::coef.
enum { CA0 = 0, CA1, CA2, CA3, CB0, CB1, CB2, CC0, CC1, CC2, CBND, CWRK1, NCOEF };

// One grid's arrays. Every pointer addresses element (0,0,0); element
// (i,j,k) is at i*S + j*P + k. All 14 arrays share P and S.
// side (nullable): the coefficients of the halo columns of the 64-cell-row
// tiles, gathered once per upload (side_index); side_kt k-tiles.
template <typename T>
struct Grid {
    const T* coef[NCOEF];
    const T* src;   // field before the iteration
    T* dst;         // wrk2
    int nx, ny, nz;
    long long P, S;
    const T* side;
    int side_kt;
};

// k-tiles of 64 own cells over an interior of nz-2 cells.
__host__ __device__ inline int kt64(int nz) { return (nz - 2 + 63) / 64; }

// Side array of the 64-cell-row tiles: for coefficient q, plane i, k-tile kt,
// row j and side s, the coefficient at column 64*kt (s = 0: the tile's
// left halo column k0-1) or 64*kt+65 (s = 1: the right one, k0+64, clamped to
// the grid). The 2*(bj+2) halo cells of a tile and plane are then 2*(bj+2)
// consecutive elements instead of as many cache lines.
__host__ __device__ inline long long side_index(int q, int i, int kt, int j, int s, int nx, int ny, int ktn)
{
    return ((((long long)q * nx + i) * ktn + kt) * ny + j) * 2 + s;
}

template <typename T>
struct Instance {
    T* f[2];            // the ping-pong pair: p buffer, wrk2 buffer
    const T* coef[NCOEF];
    int nx, ny, nz;
    long long P, S;
    int kt_n, jt_n, ichunk;
    int tile0;          // first tile of this instance in the flattened list
    const T* side;      // the instance's side array (as Grid::side)
    int side_kt;
};

// Number of i chunks of length ichunk over the interior.
__host__ __device__ inline int chunks(int nx, int ichunk) { return (nx - 2 + ichunk - 1) / ichunk; }

}  // namespace hj
