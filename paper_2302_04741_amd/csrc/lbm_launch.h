// Launcher templates: included by the per-lattice translation units, which
// instantiate them explicitly.
#pragma once

#include <algorithm>

#include "lbm_kernels.h"

namespace lbm {

inline dim3 cell_grid(const GridDims &gd, int bx)
{
    return dim3(unsigned((gd.nx + bx - 1) / bx), unsigned(gd.ny), unsigned(gd.nz));
}

// Threads per block along x: the requested count, at most nx rounded up to a
// whole wavefront.
inline int block_for(const GridDims &gd, int want)
{
    const int b = want > 0 ? want : 256;
    const int nx64 = ((gd.nx + 63) / 64) * 64;
    return b < nx64 ? b : nx64;
}

template <int LAT, class F> hipError_t with_eq_fo(int eq, int fo, F &&f)
{
    hipError_t r = hipErrorInvalidValue;
    static_for<2, Lattice<LAT>::MAXEQ + 1>([&](auto E) {
        static_for<1, 5>([&](auto O) {
            if (eq == decltype(E)::value && fo == decltype(O)::value) r = f(E, O);
        });
    });
    return r;
}

template <int LAT, class S>
hipError_t launch_step_ls(int eq, int fo, const void *A, void *B, const GridDims &gd,
                          const ForceDesc &fd, const StepCoef &co, const LaunchCfg &lc)
{
    // blocks of bx/64 wavefronts, one wavefront per 64 cells of a row
    const int64_t waves = ((int64_t(gd.nx) + 63) / 64) * gd.ny * gd.nz;
    int bx = lc.block > 0 ? lc.block : step_default_threads<LAT, S>(waves);
    bx = bx < step_max_threads<S>() ? bx : step_max_threads<S>();
    const int64_t wpb = bx / 64;
    const dim3 grid(unsigned((waves + wpb - 1) / wpb));
    return with_eq_fo<LAT>(eq, fo, [&](auto E, auto O) {
        hipLaunchKernelGGL((step_kernel<LAT, S, decltype(E)::value, decltype(O)::value>), grid,
                           dim3(bx), 0, lc.stream, static_cast<const S *>(A),
                           static_cast<S *>(B), gd, fd, co, lc.ctr, lc.cur);
        return hipGetLastError();
    });
}

template <int LAT, class S>
hipError_t launch_pattern_ls(const void *A, void *B, const GridDims &gd, const LaunchCfg &lc)
{
    // the launch shape of the step (blocks of bx/64 row wavefronts)
    const int64_t waves = ((int64_t(gd.nx) + 63) / 64) * gd.ny * gd.nz;
    int bx = lc.block > 0 ? lc.block : step_default_threads<LAT, S>(waves);
    bx = bx < step_max_threads<S>() ? bx : step_max_threads<S>();
    const int64_t wpb = bx / 64;
    hipLaunchKernelGGL((pattern_kernel<LAT, S>), dim3(unsigned((waves + wpb - 1) / wpb)),
                       dim3(bx), 0, lc.stream, static_cast<const S *>(A), static_cast<S *>(B),
                       gd);
    return hipGetLastError();
}

template <int LAT, class S>
hipError_t launch_multi_step_ls(int eq, int fo, const BatchLaunch &bl)
{
    if (bl.ntiles <= 0) return hipSuccess;
    // one wavefront per tile, or the persistent grid; the kernel strides over
    // the list, so a grid capped at 2^31 - 1 blocks still covers every tile
    const int64_t wpb = bl.threads / 64;
    const int64_t need = (bl.ntiles + wpb - 1) / wpb;
    int64_t grid = bl.blocks > 0 ? std::min(bl.blocks, need) : need;
    grid = std::min<int64_t>(grid, 0x7fffffff);
    return with_eq_fo<LAT>(eq, fo, [&](auto E, auto O) {
        constexpr int EQ = decltype(E)::value, FO = decltype(O)::value;
        if (bl.walls)
            hipLaunchKernelGGL((multi_step_kernel<LAT, S, EQ, FO, true>), dim3(unsigned(grid)),
                               dim3(unsigned(bl.threads)), 0, bl.stream, bl.begin, bl.table,
                               bl.nsims, bl.ntiles, bl.parity);
        else
            hipLaunchKernelGGL((multi_step_kernel<LAT, S, EQ, FO, false>), dim3(unsigned(grid)),
                               dim3(unsigned(bl.threads)), 0, bl.stream, bl.begin, bl.table,
                               bl.nsims, bl.ntiles, bl.parity);
        return hipGetLastError();
    });
}

template <int LAT, class S>
hipError_t launch_init_ls(int eq, int fo, const double *rho, const double *u, const double *theta,
                          void *A, const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                          const LaunchCfg &lc)
{
    const int bx = block_for(gd, 256);
    return with_eq_fo<LAT>(eq, fo, [&](auto E, auto O) {
        hipLaunchKernelGGL((init_kernel<LAT, S, decltype(E)::value, decltype(O)::value>),
                           cell_grid(gd, bx), dim3(bx), 0, lc.stream, rho, u, theta,
                           static_cast<S *>(A), gd, fd, co, lc.walls);
        return hipGetLastError();
    });
}

template <int LAT, class S>
hipError_t launch_moments_ls(const void *A, double *rho, double *u, double *theta,
                             const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                             const LaunchCfg &lc)
{
    const int bx = block_for(gd, 256);
    hipLaunchKernelGGL((moments_kernel<LAT, S>), cell_grid(gd, bx), dim3(bx), 0, lc.stream,
                       static_cast<const S *>(A), rho, u, theta, gd, fd, co, lc.walls);
    return hipGetLastError();
}

template <int LAT, class S>
hipError_t launch_heat_flux_ls(int eq, int fo, const void *A, double *q, const GridDims &gd,
                               const ForceDesc &fd, const StepCoef &co, const LaunchCfg &lc)
{
    const int bx = block_for(gd, 256);
    return with_eq_fo<LAT>(eq, fo, [&](auto E, auto O) {
        hipLaunchKernelGGL((heatflux_kernel<LAT, S, decltype(E)::value, decltype(O)::value>),
                           cell_grid(gd, bx), dim3(bx), 0, lc.stream, static_cast<const S *>(A),
                           q, gd, fd, co, lc.walls);
        return hipGetLastError();
    });
}

template <int LAT, class S>
hipError_t launch_wall_step_ls(int eq, int fo, const void *A, void *B, const GridDims &gd,
                               const ForceDesc &fd, const StepCoef &co, const LaunchCfg &lc)
{
    // the work split of the periodic step (blocks of bx/64 row wavefronts)
    const int64_t waves = ((int64_t(gd.nx) + 63) / 64) * gd.ny * gd.nz;
    int bx = lc.block > 0 ? lc.block : step_default_threads<LAT, S>(waves);
    bx = bx < step_max_threads<S>() ? bx : step_max_threads<S>();
    const int64_t wpb = bx / 64;
    const dim3 grid(unsigned((waves + wpb - 1) / wpb));
    return with_eq_fo<LAT>(eq, fo, [&](auto E, auto O) {
        hipLaunchKernelGGL((wall_step_kernel<LAT, S, decltype(E)::value, decltype(O)::value>),
                           grid, dim3(bx), 0, lc.stream, static_cast<const S *>(A),
                           static_cast<S *>(B), gd, fd, co, lc.walls, lc.ctr, lc.cur);
        return hipGetLastError();
    });
}

template <int LAT>
hipError_t launch_wall_setup_l(int eq, const double *theta, const double *uw, int64_t ny,
                               double *e, hipStream_t stream)
{
    hipError_t r = hipErrorInvalidValue;
    static_for<2, Lattice<LAT>::MAXEQ + 1>([&](auto E) {
        if (eq == decltype(E)::value) {
            hipLaunchKernelGGL((wall_setup_kernel<LAT, decltype(E)::value>), dim3(1), dim3(64), 0,
                               stream, theta[0], theta[1], uw[0], uw[1], ny, e);
            r = hipGetLastError();
        }
    });
    return r;
}

template <int LAT>
hipError_t launch_wall_mass_l(int storage, const void *A, const GridDims &gd, const StepCoef &co,
                              const LaunchCfg &lc)
{
    const int64_t ncol = int64_t(gd.nx) * gd.nz;
    const dim3 grid(unsigned((ncol + 255) / 256)), block(256);
    if (storage == 0)
        hipLaunchKernelGGL((wall_mass_kernel<LAT, double>), grid, block, 0, lc.stream,
                           static_cast<const double *>(A), gd, co, lc.walls);
    else if (storage == 1)
        hipLaunchKernelGGL((wall_mass_kernel<LAT, float>), grid, block, 0, lc.stream,
                           static_cast<const float *>(A), gd, co, lc.walls);
    else
        hipLaunchKernelGGL((wall_mass_kernel<LAT, __half>), grid, block, 0, lc.stream,
                           static_cast<const __half *>(A), gd, co, lc.walls);
    return hipGetLastError();
}

template <int LAT>
hipError_t launch_totals_l(int storage, const void *A, double *partials, double *out_dev,
                           const GridDims &gd, const StepCoef &co, hipStream_t stream)
{
    const DivU32 by_nx = make_divu32(uint32_t(gd.nx));
    if (storage == 0)
        hipLaunchKernelGGL((totals_stage1<LAT, double>), dim3(TOTALS_BLOCKS), dim3(256), 0, stream,
                           static_cast<const double *>(A), partials, gd, by_nx);
    else if (storage == 1)
        hipLaunchKernelGGL((totals_stage1<LAT, float>), dim3(TOTALS_BLOCKS), dim3(256), 0, stream,
                           static_cast<const float *>(A), partials, gd, by_nx);
    else
        hipLaunchKernelGGL((totals_stage1<LAT, __half>), dim3(TOTALS_BLOCKS), dim3(256), 0, stream,
                           static_cast<const __half *>(A), partials, gd, by_nx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((totals_stage2<LAT>), dim3(1), dim3(256), 0, stream, partials, out_dev,
                       gd, co);
    return hipGetLastError();
}

}  // namespace lbm
