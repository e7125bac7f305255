// hj_kernels.hip -- instantiation and dispatch of the sweep kernels.
#include "hj_launch.hpp"
#include "sweep_kernels.hpp"

#include <atomic>
#include <type_traits>

namespace hj {

namespace {

template <typename T> constexpr bool vec_ok(int v) { return v == 1 || v == 2 || (sizeof(T) == 4 && v == 4); }
constexpr bool bj_ok(int b) { return b == 1 || b == 2 || b == 4 || b == 8; }

template <typename T, int BJ, int V, bool NT, bool W>
hipError_t march_go(const hj_config& c, const Grid<T>& g, T omega, double* part, hipStream_t st)
{
    const TileCounts t = tile_counts(c, g.nx, g.ny, g.nz);
    const long long nb = t.tiles();
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((march_kernel<T, BJ, V, NT, W>), dim3((unsigned)nb), dim3(kWave * BJ), 0, st,
                       g, omega, c.ichunk, t.kt_n, t.jt_n, c.xcd_remap ? (int)nb : 0, part);
    return hipGetLastError();
}

template <typename T, int BJ, int V, bool NT, bool W>
hipError_t direct_go(const hj_config& c, const Grid<T>& g, T omega, double* part, hipStream_t st)
{
    const TileCounts t = tile_counts(c, g.nx, g.ny, g.nz);
    const long long nb = t.tiles();
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((direct_kernel<T, BJ, NT, W>), dim3((unsigned)nb), dim3(kWave * BJ), 0, st,
                       g, omega, t.kt_n, t.jt_n, c.xcd_remap ? (int)nb : 0, part);
    return hipGetLastError();
}

template <typename T, int BJ, int V, bool NT, bool W>
hipError_t batch_go(const Instance<T>* inst, const int* tile_inst, int ntiles, int grid,
                    int parity, T omega, double* part, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((batch_kernel<T, BJ, V, NT, W>), dim3(grid), dim3(kWave * BJ), 0, st,
                       inst, tile_inst, ntiles, parity, omega, part);
    return hipGetLastError();
}

template <typename T, int BJ, int V, bool NT>
int batch_occ()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<T, BJ, V, NT, true>,
                                                     kWave * BJ, 0) != hipSuccess)
        return 0;
    return n;
}

// Expand the run-time (bj, vec, nt, write) choice into a template instance.
#define HJ_DISPATCH_W(FN, T, BJ, V, NT, ...)                                 \
    (write ? FN<T, BJ, V, NT, true>(__VA_ARGS__) : FN<T, BJ, V, NT, false>(__VA_ARGS__))
#define HJ_DISPATCH_NT(FN, T, BJ, V, ...)                                    \
    (c.nontemporal ? HJ_DISPATCH_W(FN, T, BJ, V, true, __VA_ARGS__)          \
                   : HJ_DISPATCH_W(FN, T, BJ, V, false, __VA_ARGS__))

template <typename T, int BJ>
hipError_t march_bj(const hj_config& c, const Grid<T>& g, T omega, bool write, double* part,
                    hipStream_t st)
{
    switch (c.vec) {
    case 1: return HJ_DISPATCH_NT(march_go, T, BJ, 1, c, g, omega, part, st);
    case 2: return HJ_DISPATCH_NT(march_go, T, BJ, 2, c, g, omega, part, st);
    case 4:
        if constexpr (sizeof(T) == 4) return HJ_DISPATCH_NT(march_go, T, BJ, 4, c, g, omega, part, st);
        else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int BJ, int V>
hipError_t batch_v(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                   int grid, int parity, T omega, bool write, double* part, hipStream_t st)
{
    return HJ_DISPATCH_NT(batch_go, T, BJ, V, inst, tile_inst, ntiles, grid, parity, omega, part, st);
}

template <typename T, int BJ>
hipError_t batch_bj(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                    int grid, int parity, T omega, bool write, double* part, hipStream_t st)
{
    switch (c.vec) {
    case 1: return batch_v<T, BJ, 1>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
    case 2: return batch_v<T, BJ, 2>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
    case 4:
        if constexpr (sizeof(T) == 4)
            return batch_v<T, BJ, 4>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
        else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int BJ>
int batch_occ_bj(const hj_config& c)
{
    switch (c.vec) {
    case 1: return c.nontemporal ? batch_occ<T, BJ, 1, true>() : batch_occ<T, BJ, 1, false>();
    case 2: return c.nontemporal ? batch_occ<T, BJ, 2, true>() : batch_occ<T, BJ, 2, false>();
    case 4:
        if constexpr (sizeof(T) == 4)
            return c.nontemporal ? batch_occ<T, BJ, 4, true>() : batch_occ<T, BJ, 4, false>();
        else return 0;
    default: return 0;
    }
}

}  // namespace

bool config_supported(int dtype, const hj_config& c)
{
    if (dtype != HJ_F64 && dtype != HJ_F32) return false;
    if (c.tsteps < 0 || c.tsteps > 2 || c.reread < 0 || c.reread > 1) return false;
    if (c.xcd_remap < 0 || c.xcd_remap > 1) return false;
    if (c.tsteps == 2)
        return c.kernel == HJ_KERNEL_MARCH && c.ichunk >= 1 && c.persistent == 0 && fused_bj_ok(c.vec, c.bj);
    if (c.kernel == HJ_KERNEL_FLAT) return (c.bj == 2 || c.bj == 4 || c.bj == 8) && c.vec == 1 && c.ichunk >= 1;
    if (!bj_ok(c.bj)) return false;
    if (c.kernel == HJ_KERNEL_DIRECT) return c.bj >= 2;
    if (c.kernel != HJ_KERNEL_MARCH) return false;
    if (c.ichunk < 1) return false;
    return dtype == HJ_F64 ? vec_ok<double>(c.vec) : vec_ok<float>(c.vec);
}

bool config_fits(int dtype, const hj_config& c, int nx, int ny, int nz)
{
    (void)nx;
    if (!config_supported(dtype, c)) return false;
    const int esz = dtype == HJ_F64 ? 8 : 4;
    if (c.kernel == HJ_KERNEL_FLAT) return flat_fits(esz, c.bj, ny, nz);
    if (fused_of(c)) return plane32_ok(esz, ny, nz);
    return true;
}

namespace {

template <typename T, int NW, int V, bool NT, bool W>
hipError_t flat_go(const hj_config& c, const Grid<T>& g, T omega, double* part, hipStream_t st)
{
    static_assert(kFlatPlaneBytes == kFlatPlaneBytesHost, "flat plane size");
    if (!flat_fits((int)sizeof(T), NW, g.ny, g.nz)) return hipErrorInvalidValue;
    const TileCounts t = tile_counts(c, g.nx, g.ny, g.nz);
    const long long nb = t.tiles();
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((flat_kernel<T, NW, NT, W>), dim3((unsigned)nb), dim3(kWave * NW), 0, st, g, omega,
                       c.ichunk, t.kt_n, c.xcd_remap ? (int)nb : 0, part);
    return hipGetLastError();
}

template <typename T, int NW, int V, bool NT, bool W>
hipError_t flat_batch_go(const Instance<T>* inst, const int* tile_inst, int ntiles, int grid, int parity,
                         T omega, double* part, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((flat_batch_kernel<T, NW, NT, W>), dim3(grid), dim3(kWave * NW), 0, st, inst, tile_inst,
                       ntiles, parity, omega, part);
    return hipGetLastError();
}

template <typename T, int NW, bool NT>
int flat_batch_occ()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, flat_batch_kernel<T, NW, NT, true>, kWave * NW, 0) !=
        hipSuccess)
        return 0;
    return n;
}

}  // namespace

template <typename T>
hipError_t launch_sweep(const hj_config& c, const Grid<T>& g, T omega, bool write, double* part,
                        hipStream_t st)
{
    if (fused_of(c)) return hipErrorInvalidValue;
    if (c.kernel == HJ_KERNEL_FLAT) {
        switch (c.bj) {
        case 2: return HJ_DISPATCH_NT(flat_go, T, 2, 1, c, g, omega, part, st);
        case 4: return HJ_DISPATCH_NT(flat_go, T, 4, 1, c, g, omega, part, st);
        case 8: return HJ_DISPATCH_NT(flat_go, T, 8, 1, c, g, omega, part, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (c.kernel == HJ_KERNEL_DIRECT) {
        switch (c.bj) {
        case 2: return HJ_DISPATCH_NT(direct_go, T, 2, 1, c, g, omega, part, st);
        case 4: return HJ_DISPATCH_NT(direct_go, T, 4, 1, c, g, omega, part, st);
        case 8: return HJ_DISPATCH_NT(direct_go, T, 8, 1, c, g, omega, part, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (c.bj) {
    case 1: return march_bj<T, 1>(c, g, omega, write, part, st);
    case 2: return march_bj<T, 2>(c, g, omega, write, part, st);
    case 4: return march_bj<T, 4>(c, g, omega, write, part, st);
    case 8: return march_bj<T, 8>(c, g, omega, write, part, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_batch(const hj_config& c, const Instance<T>* inst, const int* tile_inst,
                        int ntiles, int grid, int parity, T omega, bool write, double* part,
                        hipStream_t st)
{
    if (c.kernel == HJ_KERNEL_FLAT) {
        switch (c.bj) {
        case 2: return HJ_DISPATCH_NT(flat_batch_go, T, 2, 1, inst, tile_inst, ntiles, grid, parity, omega, part, st);
        case 4: return HJ_DISPATCH_NT(flat_batch_go, T, 4, 1, inst, tile_inst, ntiles, grid, parity, omega, part, st);
        case 8: return HJ_DISPATCH_NT(flat_batch_go, T, 8, 1, inst, tile_inst, ntiles, grid, parity, omega, part, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (c.bj) {
    case 1: return batch_bj<T, 1>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
    case 2: return batch_bj<T, 2>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
    case 4: return batch_bj<T, 4>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
    case 8: return batch_bj<T, 8>(c, inst, tile_inst, ntiles, grid, parity, omega, write, part, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
int batch_occupancy(const hj_config& c)
{
    if (c.kernel == HJ_KERNEL_FLAT) {
        switch (c.bj) {
        case 2: return c.nontemporal ? flat_batch_occ<T, 2, true>() : flat_batch_occ<T, 2, false>();
        case 4: return c.nontemporal ? flat_batch_occ<T, 4, true>() : flat_batch_occ<T, 4, false>();
        case 8: return c.nontemporal ? flat_batch_occ<T, 8, true>() : flat_batch_occ<T, 8, false>();
        default: return 0;
        }
    }
    switch (c.bj) {
    case 1: return batch_occ_bj<T, 1>(c);
    case 2: return batch_occ_bj<T, 2>(c);
    case 4: return batch_occ_bj<T, 4>(c);
    case 8: return batch_occ_bj<T, 8>(c);
    default: return 0;
    }
}

namespace {

// The remap window of a single-grid two-iteration launch (see remap_xcd):
// the workgroups of `kernel` resident on the current device at once, a
// multiple of 8; 0 without the remap. Queried once per kernel and device:
// `cache` is the kernel's own table (one entry per device, 0 until queried).
constexpr int kMaxDevices = 64;
template <typename K>
int remap_window(const hj_config& c, K kernel, int threads, std::atomic<int>* cache)
{
    if (!c.xcd_remap) return 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int w = cache[dev].load(std::memory_order_relaxed);
    if (w == 0) {
        int occ = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess) occ = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
        w = occ * cus / 8 * 8;
        if (w <= 0) w = 0x7fffffff;  // no answer: deal the whole grid, as with one window
        cache[dev].store(w, std::memory_order_relaxed);
    }
    return w;
}

// Each two-iteration single-grid kernel's table of remap windows (one entry
// per device), shared by its launcher and prime_remap.
template <typename T, int BJ, int W, bool NT, bool KEEP>
std::atomic<int>* fused_win()
{
    static std::atomic<int> c[kMaxDevices];
    return c;
}
template <typename T, int BJ, bool NT, bool KEEP>
std::atomic<int>* wide_win()
{
    static std::atomic<int> c[kMaxDevices];
    return c;
}

template <typename T, int BJ, int W, bool NT, bool KEEP>
hipError_t fused_go(const hj_config& c, const Grid<T>& g, T omega, double* part1, double* part2,
                    hipStream_t st)
{
    if (!plane32_ok((int)sizeof(T), g.ny, g.nz)) return hipErrorInvalidValue;  // 32-bit plane offsets
    const TileCounts t = tile_counts(c, g.nx, g.ny, g.nz);
    const long long nb = t.tiles();
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    const int win =
        remap_window(c, fused_kernel<T, BJ, W, NT, KEEP>, fused_threads<BJ, W>(), fused_win<T, BJ, W, NT, KEEP>());
    hipLaunchKernelGGL((fused_kernel<T, BJ, W, NT, KEEP>), dim3((unsigned)nb), dim3(fused_threads<BJ, W>()), 0, st,
                       g, omega, c.ichunk, t.kt_n, t.jt_n, win, part1, part2);
    return hipGetLastError();
}

template <typename T, int BJ, int W, bool NT, bool KEEP>
hipError_t fused_batch_go(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                          int parity, T omega, double* part1, double* part2, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    // a batch deals its whole tile list in eighths: each XCD keeps whole instances in its L2
    const int win = c.xcd_remap ? ntiles : 0;
    hipLaunchKernelGGL((fused_batch_kernel<T, BJ, W, NT, KEEP>), dim3((unsigned)ntiles),
                       dim3(fused_threads<BJ, W>()), 0, st, inst, tile_inst, parity, omega, win, part1, part2);
    return hipGetLastError();
}

template <typename T, int BJ, bool NT, bool KEEP>
hipError_t wide_go(const hj_config& c, const Grid<T>& g, T omega, double* part1, double* part2, hipStream_t st)
{
    if (!plane32_ok((int)sizeof(T), g.ny, g.nz)) return hipErrorInvalidValue;  // 32-bit plane offsets
    // the prefetching form reads the halo columns' coefficients from the side array
    if (prefetch_wide<T>(BJ) > 0 && (!g.side || g.side_kt != kt64(g.nz))) return hipErrorInvalidValue;
    const TileCounts t = tile_counts(c, g.nx, g.ny, g.nz);
    const long long nb = t.tiles();
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    const int win = remap_window(c, wide_kernel<T, BJ, NT, KEEP>, kWave * (BJ + 3), wide_win<T, BJ, NT, KEEP>());
    hipLaunchKernelGGL((wide_kernel<T, BJ, NT, KEEP>), dim3((unsigned)nb), dim3(kWave * (BJ + 3)), 0, st, g, omega,
                       c.ichunk, t.kt_n, t.jt_n, win, part1, part2);
    return hipGetLastError();
}

template <typename T, int BJ, bool NT, bool KEEP>
hipError_t wide_batch_go(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                         int parity, T omega, double* part1, double* part2, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const int win = c.xcd_remap ? ntiles : 0;  // as for fused_batch_go
    hipLaunchKernelGGL((wide_batch_kernel<T, BJ, NT, KEEP>), dim3((unsigned)ntiles), dim3(kWave * (BJ + 3)), 0,
                       st, inst, tile_inst, parity, omega, win, part1, part2);
    return hipGetLastError();
}

// Calls f(nt, keep) with std::bool_constant arguments for the streaming
// mode (nontemporal) and coefficient mode (KEEP = !reread) of c.
template <typename F>
auto with_modes(const hj_config& c, F&& f)
{
    if (c.reread) return c.nontemporal ? f(std::true_type{}, std::false_type{}) : f(std::false_type{}, std::false_type{});
    return c.nontemporal ? f(std::true_type{}, std::true_type{}) : f(std::false_type{}, std::true_type{});
}

template <typename T, int BJ>
hipError_t fused_batch_bj(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                          int parity, T omega, double* part1, double* part2, hipStream_t st)
{
    return with_modes(c, [&](auto nt, auto keep) -> hipError_t {
        constexpr bool NT = decltype(nt)::value, KEEP = decltype(keep)::value;
        if (c.vec == 1) {
            if constexpr (fused_bj_ok(1, BJ))
                return fused_batch_go<T, BJ, kWave, NT, KEEP>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
        } else if (c.vec == 2) {
            if constexpr (fused_bj_ok(2, BJ))
                return wide_batch_go<T, BJ, NT, KEEP>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
        } else if (c.vec == 4) {
            if constexpr (fused_bj_ok(4, BJ))
                return fused_batch_go<T, BJ, kWave / 2, NT, KEEP>(c, inst, tile_inst, ntiles, parity, omega, part1,
                                                                 part2, st);
        }
        return hipErrorInvalidValue;
    });
}

template <typename T, int BJ>
hipError_t fused_bj(const hj_config& c, const Grid<T>& g, T omega, double* part1, double* part2,
                    hipStream_t st)
{
    return with_modes(c, [&](auto nt, auto keep) -> hipError_t {
        constexpr bool NT = decltype(nt)::value, KEEP = decltype(keep)::value;
        if (c.vec == 1) {
            if constexpr (fused_bj_ok(1, BJ)) return fused_go<T, BJ, kWave, NT, KEEP>(c, g, omega, part1, part2, st);
        } else if (c.vec == 2) {
            if constexpr (fused_bj_ok(2, BJ)) return wide_go<T, BJ, NT, KEEP>(c, g, omega, part1, part2, st);
        } else if (c.vec == 4) {
            if constexpr (fused_bj_ok(4, BJ))
                return fused_go<T, BJ, kWave / 2, NT, KEEP>(c, g, omega, part1, part2, st);
        }
        return hipErrorInvalidValue;
    });
}

template <typename T, int BJ>
int fused_occ_bj(const hj_config& c)
{
    return with_modes(c, [&](auto nt, auto keep) -> int {
        constexpr bool NT = decltype(nt)::value, KEEP = decltype(keep)::value;
        int n = 0;
        hipError_t e = hipErrorInvalidValue;
        if (c.vec == 1) {
            if constexpr (fused_bj_ok(1, BJ))
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fused_kernel<T, BJ, kWave, NT, KEEP>,
                                                                 fused_threads<BJ, kWave>(), 0);
        } else if (c.vec == 2) {
            if constexpr (fused_bj_ok(2, BJ))
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wide_kernel<T, BJ, NT, KEEP>, kWave * (BJ + 3), 0);
        } else if (c.vec == 4) {
            if constexpr (fused_bj_ok(4, BJ))
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fused_kernel<T, BJ, kWave / 2, NT, KEEP>,
                                                                 fused_threads<BJ, kWave / 2>(), 0);
        }
        return e == hipSuccess ? n : 0;
    });
}

}  // namespace

template <typename T>
int fused_occupancy(const hj_config& c)
{
    if (!fused_of(c)) return 0;
    switch (c.bj) {
    case 2: return fused_occ_bj<T, 2>(c);
    case 4: return fused_occ_bj<T, 4>(c);
    case 6: return fused_occ_bj<T, 6>(c);
    case 8: return fused_occ_bj<T, 8>(c);
    case 12: return fused_occ_bj<T, 12>(c);
    case 14: return fused_occ_bj<T, 14>(c);
    case 22: return fused_occ_bj<T, 22>(c);
    case 30: return fused_occ_bj<T, 30>(c);
    default: return 0;
    }
}

template int fused_occupancy<double>(const hj_config&);
template int fused_occupancy<float>(const hj_config&);

namespace {

template <typename T, int BJ>
void prime_bj(const hj_config& c)
{
    with_modes(c, [&](auto nt, auto keep) -> int {
        constexpr bool NT = decltype(nt)::value, KEEP = decltype(keep)::value;
        if (c.vec == 1) {
            if constexpr (fused_bj_ok(1, BJ))
                (void)remap_window(c, fused_kernel<T, BJ, kWave, NT, KEEP>, fused_threads<BJ, kWave>(),
                                   fused_win<T, BJ, kWave, NT, KEEP>());
        } else if (c.vec == 2) {
            if constexpr (fused_bj_ok(2, BJ))
                (void)remap_window(c, wide_kernel<T, BJ, NT, KEEP>, kWave * (BJ + 3), wide_win<T, BJ, NT, KEEP>());
        } else if (c.vec == 4) {
            if constexpr (fused_bj_ok(4, BJ))
                (void)remap_window(c, fused_kernel<T, BJ, kWave / 2, NT, KEEP>, fused_threads<BJ, kWave / 2>(),
                                   fused_win<T, BJ, kWave / 2, NT, KEEP>());
        }
        return 0;
    });
}

}  // namespace

template <typename T>
void prime_remap(const hj_config& c)
{
    if (c.tsteps != 2 || !c.xcd_remap || !fused_bj_ok(c.vec, c.bj)) return;
    switch (c.bj) {
    case 2: prime_bj<T, 2>(c); break;
    case 4: prime_bj<T, 4>(c); break;
    case 6: prime_bj<T, 6>(c); break;
    case 8: prime_bj<T, 8>(c); break;
    case 12: prime_bj<T, 12>(c); break;
    case 14: prime_bj<T, 14>(c); break;
    case 22: prime_bj<T, 22>(c); break;
    case 30: prime_bj<T, 30>(c); break;
    default: break;
    }
}

template void prime_remap<double>(const hj_config&);
template void prime_remap<float>(const hj_config&);

template <typename T>
hipError_t launch_fused(const hj_config& c, const Grid<T>& g, T omega, double* part1, double* part2,
                        hipStream_t st)
{
    if (!fused_of(c) || c.kernel != HJ_KERNEL_MARCH || !fused_bj_ok(c.vec, c.bj) || c.ichunk < 1)
        return hipErrorInvalidValue;
    switch (c.bj) {
    case 2: return fused_bj<T, 2>(c, g, omega, part1, part2, st);
    case 4: return fused_bj<T, 4>(c, g, omega, part1, part2, st);
    case 6: return fused_bj<T, 6>(c, g, omega, part1, part2, st);
    case 8: return fused_bj<T, 8>(c, g, omega, part1, part2, st);
    case 12: return fused_bj<T, 12>(c, g, omega, part1, part2, st);
    case 14: return fused_bj<T, 14>(c, g, omega, part1, part2, st);
    case 22: return fused_bj<T, 22>(c, g, omega, part1, part2, st);
    case 30: return fused_bj<T, 30>(c, g, omega, part1, part2, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_batch_fused(const hj_config& c, const Instance<T>* inst, const int* tile_inst, int ntiles,
                              int parity, T omega, double* part1, double* part2, hipStream_t st)
{
    if (!fused_of(c) || c.kernel != HJ_KERNEL_MARCH || !fused_bj_ok(c.vec, c.bj) || c.ichunk < 1 || c.persistent)
        return hipErrorInvalidValue;
    switch (c.bj) {
    case 2: return fused_batch_bj<T, 2>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 4: return fused_batch_bj<T, 4>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 6: return fused_batch_bj<T, 6>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 8: return fused_batch_bj<T, 8>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 12: return fused_batch_bj<T, 12>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 14: return fused_batch_bj<T, 14>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 22: return fused_batch_bj<T, 22>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    case 30: return fused_batch_bj<T, 30>(c, inst, tile_inst, ntiles, parity, omega, part1, part2, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_batch_fused<double>(const hj_config&, const Instance<double>*, const int*, int, int,
                                               double, double*, double*, hipStream_t);
template hipError_t launch_batch_fused<float>(const hj_config&, const Instance<float>*, const int*, int, int,
                                              float, double*, double*, hipStream_t);

template hipError_t launch_fused<double>(const hj_config&, const Grid<double>&, double, double*, double*,
                                         hipStream_t);
template hipError_t launch_fused<float>(const hj_config&, const Grid<float>&, float, double*, double*,
                                        hipStream_t);

template hipError_t launch_sweep<double>(const hj_config&, const Grid<double>&, double, bool,
                                         double*, hipStream_t);
template hipError_t launch_sweep<float>(const hj_config&, const Grid<float>&, float, bool, double*,
                                        hipStream_t);
template hipError_t launch_batch<double>(const hj_config&, const Instance<double>*, const int*, int,
                                         int, int, double, bool, double*, hipStream_t);
template hipError_t launch_batch<float>(const hj_config&, const Instance<float>*, const int*, int,
                                        int, int, float, bool, double*, hipStream_t);
template int batch_occupancy<double>(const hj_config&);
template int batch_occupancy<float>(const hj_config&);

hipError_t launch_finalize(const double* part, long long stride, int n, const int* seg_begin,
                           int nseg, int nslots, double* out, hipStream_t st)
{
    if (nslots <= 0 || nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(nseg, nslots), dim3(256), 0, st, part, stride, n,
                       seg_begin, nseg, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_side_gather(const T* coef, T* side, int nx, int ny, int nz, long long P, long long S,
                              hipStream_t st)
{
    const int ktn = kt64(nz);
    const long long n = (long long)nx * ktn * ny * 2;
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((side_gather_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, coef, side, nx, ny, nz, P, S,
                       ktn);
    return hipGetLastError();
}

template hipError_t launch_side_gather<double>(const double*, double*, int, int, int, long long, long long,
                                               hipStream_t);
template hipError_t launch_side_gather<float>(const float*, float*, int, int, int, long long, long long,
                                              hipStream_t);

hipError_t launch_copy(void* dst, const void* src, unsigned long long bytes, hipStream_t st)
{
    const long long n16 = (long long)(bytes / 16);
    if (n16 <= 0) return hipSuccess;
    long long blocks = (n16 + 255) / 256;
    if (blocks > 256LL * 32) blocks = 256LL * 32;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const u32x4*>(src), reinterpret_cast<u32x4*>(dst), n16);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stream_probe(const Grid<T>& g, int vec, int ichunk, hipStream_t st)
{
    constexpr int BJ = 4;
    if (ichunk < 1) return hipErrorInvalidValue;
    const int V = (vec == 4 && sizeof(T) == 4) ? 4 : (vec == 2 ? 2 : 1);
    const int kt_n = (g.nz - 2 + kWave * V - 1) / (kWave * V);
    const int jt_n = (g.ny - 2 + BJ - 1) / BJ;
    const long long nb = (long long)kt_n * jt_n * chunks(g.nx, ichunk);
    if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (V == 4) {
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((stream_kernel<T, BJ, 4>), dim3((unsigned)nb), dim3(kWave * BJ), 0, st, g, ichunk, kt_n, jt_n);
    } else if (V == 2) {
        hipLaunchKernelGGL((stream_kernel<T, BJ, 2>), dim3((unsigned)nb), dim3(kWave * BJ), 0, st, g, ichunk, kt_n, jt_n);
    } else {
        hipLaunchKernelGGL((stream_kernel<T, BJ, 1>), dim3((unsigned)nb), dim3(kWave * BJ), 0, st, g, ichunk, kt_n, jt_n);
    }
    return hipGetLastError();
}

template hipError_t launch_stream_probe<double>(const Grid<double>&, int, int, hipStream_t);
template hipError_t launch_stream_probe<float>(const Grid<float>&, int, int, hipStream_t);

hipError_t launch_diff(const void* a, const void* b, unsigned long long bytes,
                       unsigned long long* count, hipStream_t st)
{
    const long long n4 = (long long)(bytes / 4);
    if (n4 <= 0) return hipSuccess;
    long long blocks = (n4 + 255) / 256;
    if (blocks > 256LL * 16) blocks = 256LL * 16;
    hipLaunchKernelGGL(diff_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const uint32_t*>(a), reinterpret_cast<const uint32_t*>(b),
                       n4, count);
    return hipGetLastError();
}

}  // namespace hj
