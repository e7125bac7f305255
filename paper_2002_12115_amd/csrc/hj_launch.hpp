// hj_launch.hpp -- host-side launchers of the sweep kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/hj.h"
#include "sweep_types.hpp"

namespace hj {

struct TileCounts {
    int kt_n, jt_n, ic_n;
    long long tiles() const { return (long long)kt_n * jt_n * ic_n; }
};

inline int vec_of(const hj_config& c) { return c.kernel == HJ_KERNEL_DIRECT ? 1 : c.vec; }

inline bool fused_of(const hj_config& c) { return c.tsteps == 2; }

// Row layouts of the two-iteration kernels (hj_config::vec when tsteps is 2):
// 1: one 64-lane row per wave, 62 own cells; 2: 64 own cells per row with a
// halo wave beside the rows; 4: two 32-lane rows per wave, 30 own cells.
// Own k cells per tile:
inline int fused_tk(const hj_config& c) { return c.vec == 2 ? kWave : c.vec == 4 ? kWave / 2 - 2 : kWave - 2; }

// The bj (own rows per tile) each layout is built for: the workgroup is
// bj+2 waves (layout 1), bj+3 waves (layout 2) or (bj+2)/2 waves (layout 4).
constexpr bool fused_bj_ok(int vec, int bj)
{
    return vec == 1   ? (bj == 2 || bj == 4 || bj == 6 || bj == 8 || bj == 14)
           : vec == 2 ? (bj == 2 || bj == 4 || bj == 6 || bj == 8 || bj == 12)
           : vec == 4 ? (bj == 6 || bj == 14 || bj == 22 || bj == 30)
                      : false;
}

// Pitch of a k row in elements: a front pad of A-1 elements (A = 128 B of
// elements) puts interior k=1 on a 128-byte boundary; the row, with 4 spare
// elements, is rounded up to a multiple of A.
inline long long pitch_of(int esz, int nz)
{
    const long long A = 128 / esz;
    return (A + nz + 4 + A - 1) / A * A;
}

// The prefetching two-iteration kernels address a plane with 32-bit byte
// offsets: a plane (ny rows of the pitch) must hold fewer than 2^32 bytes.
// Two-iteration configurations are refused for larger planes in both dtypes.
inline bool plane32_ok(int esz, int ny, int nz)
{
    return (long long)ny * pitch_of(esz, nz) * esz < (1LL << 32);
}

// LDS bytes per staged plane of the flat kernel.
constexpr int kFlatPlaneBytesHost = 10240;

// Whether the flat kernel with 64*nw-cell runs fits a grid: the rows a run
// touches, plus its halo rows, times nz, must fit one staged plane.
inline bool flat_fits(int esz, int nw, int ny, int nz)
{
    const long long nzi = nz - 2, t = 64LL * nw;
    long long rows = (t - 1 + nzi - 1) / nzi + 3;
    if (rows > ny) rows = ny;
    return rows * nz <= kFlatPlaneBytesHost / esz;
}

inline TileCounts tile_counts(const hj_config& c, int nx, int ny, int nz)
{
    TileCounts t;
    if (fused_of(c)) {
        const int tk = fused_tk(c);
        t.kt_n = (nz - 2 + tk - 1) / tk;
        t.jt_n = (ny - 2 + c.bj - 1) / c.bj;
        t.ic_n = chunks(nx, c.ichunk);
        return t;
    }
    if (c.kernel == HJ_KERNEL_FLAT) {
        const long long cells = (long long)(ny - 2) * (nz - 2);
        t.kt_n = (int)((cells + 64LL * c.bj - 1) / (64LL * c.bj));
        t.jt_n = 1;
        t.ic_n = chunks(nx, c.ichunk);
        return t;
    }
    const int tk = kWave * vec_of(c);
    t.kt_n = (nz - 2 + tk - 1) / tk;
    t.jt_n = (ny - 2 + c.bj - 1) / c.bj;
    t.ic_n = c.kernel == HJ_KERNEL_DIRECT ? nx - 2 : chunks(nx, c.ichunk);
    return t;
}

// True when (dtype, config) names an instantiated kernel.
bool config_supported(int dtype, const hj_config& c);

// True when the configuration is supported and can run this grid.
bool config_fits(int dtype, const hj_config& c, int nx, int ny, int nz);

// One sweep (write) or residual (no write) over a single grid. part receives
// one FP64 partial per tile (tile_counts(...).tiles() of them).
template <typename T>
hipError_t launch_sweep(const hj_config& c, const Grid<T>& g, T omega, bool write, double* part,
                        hipStream_t st);

// Two iterations over a single grid (tsteps 2): g.src -> g.dst, with the
// first iteration's per-tile gosa partials to part1 and the second's to part2.
template <typename T>
hipError_t launch_fused(const hj_config& c, const Grid<T>& g, T omega, double* part1, double* part2,
                        hipStream_t st);

// Two iterations over every instance of a batch (tsteps 2, not persistent):
// one workgroup per tile of the flattened list, built with the two-iteration
// tile counts; tile_inst holds 2*ntiles ints, (instance, tile within the
// instance) in dispatch order; per-tile partials of the two iterations to
// part1 and part2 at the tiles' instance-major places.
template <typename T>
hipError_t launch_batch_fused(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                              int parity, T omega, double* part1, double* part2, hipStream_t st);

// Query, outside any stream capture, what the launch of c's single-grid
// two-iteration kernel on the current device will ask the runtime (its XCD
// remap window), so that later launches, captured ones included, make no
// runtime query. Does nothing for other configurations.
template <typename T>
void prime_remap(const hj_config& c);

// Workgroups of the two-iteration kernel named by c resident per CU (0 when
// c names none, or the query fails).
template <typename T>
int fused_occupancy(const hj_config& c);

// One iteration over every instance of a batch.
template <typename T>
hipError_t launch_batch(const hj_config& c, const Instance<T>* inst, const int* tile_inst,
                        int ntiles, int grid, int parity, T omega, bool write, double* part,
                        hipStream_t st);

// Workgroups per CU the batch kernel of this configuration can keep resident.
template <typename T>
int batch_occupancy(const hj_config& c);

hipError_t launch_finalize(const double* part, long long stride, int n, const int* seg_begin,
                           int nseg, int nslots, double* out, hipStream_t st);

hipError_t launch_copy(void* dst, const void* src, unsigned long long bytes, hipStream_t st);

// Fill coefficient q's block of a solve's side array (see side_index) from
// the coefficient's field: coef addresses element (0,0,0), side the block.
template <typename T>
hipError_t launch_side_gather(const T* coef, T* side, int nx, int ny, int nz, long long P, long long S,
                              hipStream_t st);

// 13-read / 1-write streaming probe over the interior (bj 4, V = 1 or 4).
template <typename T>
hipError_t launch_stream_probe(const Grid<T>& g, int vec, int ichunk, hipStream_t st);

hipError_t launch_diff(const void* a, const void* b, unsigned long long bytes,
                       unsigned long long* count, hipStream_t st);

}  // namespace hj
