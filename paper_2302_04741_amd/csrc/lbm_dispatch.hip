// Generic launchers: switch on lattice and storage to the per-lattice pieces.
#include "lbm_internal.h"

namespace lbm {

namespace {
template <class T>
__global__ void __launch_bounds__(256) convert_kernel(const double *__restrict__ src,
                                                      T *__restrict__ dst, int64_t n)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = T(src[k]);
}
}  // namespace

hipError_t launch_step(int lat, int storage, int eq, int fo, const void *A, void *B,
                       const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                       const LaunchCfg &lc)
{
    if (lat == 0 && storage == 0) return launch_step_ls<0, double>(eq, fo, A, B, gd, fd, co, lc);
    if (lat == 0 && storage == 1) return launch_step_ls<0, float>(eq, fo, A, B, gd, fd, co, lc);
    if (lat == 1 && storage == 0) return launch_step_ls<1, double>(eq, fo, A, B, gd, fd, co, lc);
    if (lat == 1 && storage == 1) return launch_step_ls<1, float>(eq, fo, A, B, gd, fd, co, lc);
    if (lat == 0 && storage == 2) return launch_step_ls<0, __half>(eq, fo, A, B, gd, fd, co, lc);
    if (lat == 1 && storage == 2) return launch_step_ls<1, __half>(eq, fo, A, B, gd, fd, co, lc);
    return hipErrorInvalidValue;
}

hipError_t launch_pattern(int lat, int storage, const void *A, void *B, const GridDims &gd,
                          const LaunchCfg &lc)
{
    if (lat == 0 && storage == 0) return launch_pattern_ls<0, double>(A, B, gd, lc);
    if (lat == 0 && storage == 1) return launch_pattern_ls<0, float>(A, B, gd, lc);
    if (lat == 1 && storage == 0) return launch_pattern_ls<1, double>(A, B, gd, lc);
    if (lat == 1 && storage == 1) return launch_pattern_ls<1, float>(A, B, gd, lc);
    if (lat == 0 && storage == 2) return launch_pattern_ls<0, __half>(A, B, gd, lc);
    if (lat == 1 && storage == 2) return launch_pattern_ls<1, __half>(A, B, gd, lc);
    return hipErrorInvalidValue;
}

hipError_t launch_wall_setup(int lat, int eq, const double *theta, const double *uw, int64_t ny,
                             double *e, hipStream_t stream)
{
    if (lat == 0) return launch_wall_setup_l<0>(eq, theta, uw, ny, e, stream);
    if (lat == 1) return launch_wall_setup_l<1>(eq, theta, uw, ny, e, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_wall_mass(int lat, int storage, const void *A, const GridDims &gd,
                            const StepCoef &co, const LaunchCfg &lc)
{
    if (lat == 0) return launch_wall_mass_l<0>(storage, A, gd, co, lc);
    if (lat == 1) return launch_wall_mass_l<1>(storage, A, gd, co, lc);
    return hipErrorInvalidValue;
}

hipError_t launch_wall_step(int lat, int storage, int eq, int fo, const void *A, void *B,
                            const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                            const LaunchCfg &lc)
{
#define LBM_WS(L, S) return launch_wall_step_ls<L, S>(eq, fo, A, B, gd, fd, co, lc)
    if (lat == 0 && storage == 0) LBM_WS(0, double);
    if (lat == 0 && storage == 1) LBM_WS(0, float);
    if (lat == 0 && storage == 2) LBM_WS(0, __half);
    if (lat == 1 && storage == 0) LBM_WS(1, double);
    if (lat == 1 && storage == 1) LBM_WS(1, float);
    if (lat == 1 && storage == 2) LBM_WS(1, __half);
#undef LBM_WS
    return hipErrorInvalidValue;
}

hipError_t launch_multi_step(int lat, int storage, int eq, int fo, const BatchLaunch &bl)
{
#define LBM_MS(L, S) return launch_multi_step_ls<L, S>(eq, fo, bl)
    if (lat == 0 && storage == 0) LBM_MS(0, double);
    if (lat == 0 && storage == 1) LBM_MS(0, float);
    if (lat == 0 && storage == 2) LBM_MS(0, __half);
    if (lat == 1 && storage == 0) LBM_MS(1, double);
    if (lat == 1 && storage == 1) LBM_MS(1, float);
    if (lat == 1 && storage == 2) LBM_MS(1, __half);
#undef LBM_MS
    return hipErrorInvalidValue;
}

#define LBM_BY_STORAGE(CALL)                                   \
    if (lat == 0 && storage == 0) return CALL(0, double);      \
    if (lat == 0 && storage == 1) return CALL(0, float);       \
    if (lat == 0 && storage == 2) return CALL(0, __half);      \
    if (lat == 1 && storage == 0) return CALL(1, double);      \
    if (lat == 1 && storage == 1) return CALL(1, float);       \
    if (lat == 1 && storage == 2) return CALL(1, __half);      \
    return hipErrorInvalidValue

hipError_t launch_init(int lat, int storage, int eq, int fo, const double *rho, const double *u,
                       const double *theta, void *A, const GridDims &gd, const ForceDesc &fd,
                       const StepCoef &co, const LaunchCfg &lc)
{
#define LBM_INIT(L, S) launch_init_ls<L, S>(eq, fo, rho, u, theta, A, gd, fd, co, lc)
    LBM_BY_STORAGE(LBM_INIT);
#undef LBM_INIT
}

hipError_t launch_moments(int lat, int storage, const void *A, double *rho, double *u,
                          double *theta, const GridDims &gd, const ForceDesc &fd,
                          const StepCoef &co, const LaunchCfg &lc)
{
#define LBM_MOM(L, S) launch_moments_ls<L, S>(A, rho, u, theta, gd, fd, co, lc)
    LBM_BY_STORAGE(LBM_MOM);
#undef LBM_MOM
}

hipError_t launch_heat_flux(int lat, int storage, int eq, int fo, const void *A, double *q,
                            const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                            const LaunchCfg &lc)
{
#define LBM_HF(L, S) launch_heat_flux_ls<L, S>(eq, fo, A, q, gd, fd, co, lc)
    LBM_BY_STORAGE(LBM_HF);
#undef LBM_HF
}

#undef LBM_BY_STORAGE

hipError_t launch_totals(int lat, int storage, const void *A, double *partials, double *out_dev,
                         const GridDims &gd, const StepCoef &co, hipStream_t stream)
{
    if (lat == 0) return launch_totals_l<0>(storage, A, partials, out_dev, gd, co, stream);
    if (lat == 1) return launch_totals_l<1>(storage, A, partials, out_dev, gd, co, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_convert(int storage, const double *src, void *dst, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const unsigned nb = unsigned((n + 255) / 256);
    if (storage == 0)
        hipLaunchKernelGGL((convert_kernel<double>), dim3(nb), dim3(256), 0, stream, src,
                           static_cast<double *>(dst), n);
    else
        hipLaunchKernelGGL((convert_kernel<float>), dim3(nb), dim3(256), 0, stream, src,
                           static_cast<float *>(dst), n);
    return hipGetLastError();
}

}  // namespace lbm
