// sweep_types.hpp -- data types shared by the sweep kernels and the runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace hj {

constexpr int kWave = 64;

// Coefficient slots inside Grid::coef.
enum { CA0 = 0, CA1, CA2, CA3, CB0, CB1, CB2, CC0, CC1, CC2, CBND, CWRK1, NCOEF };

// One grid's arrays. Every pointer addresses element (0,0,0); element
// (i,j,k) is at i*S + j*P + k. All 14 arrays share P and S.
template <typename T>
struct Grid {
    const T* coef[NCOEF];
    const T* src;   // field before the iteration
    T* dst;         // wrk2
    int nx, ny, nz;
    long long P, S;
};

template <typename T>
struct Instance {
    T* f[2];            // the ping-pong pair: p buffer, wrk2 buffer
    const T* coef[NCOEF];
    int nx, ny, nz;
    long long P, S;
    int kt_n, jt_n, ichunk;
    int tile0;          // first tile of this instance in the flattened list
};

// Number of i chunks of length ichunk over the interior.
__host__ __device__ inline int chunks(int nx, int ichunk) { return (nx - 2 + ichunk - 1) / ichunk; }

}  // namespace hj
