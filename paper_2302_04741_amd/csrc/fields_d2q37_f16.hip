// Initialisation, moments and heat-flux kernels for D2Q37 storage f16 (all orders).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_init_ls<0, __half>(int, int, const double *, const double *,
                                               const double *, void *, const GridDims &,
                                               const ForceDesc &, const StepCoef &,
                                               const LaunchCfg &);
template hipError_t launch_moments_ls<0, __half>(const void *, double *, double *, double *,
                                                  const GridDims &, const ForceDesc &,
                                                  const StepCoef &, const LaunchCfg &);
template hipError_t launch_heat_flux_ls<0, __half>(int, int, const void *, double *,
                                                    const GridDims &, const ForceDesc &,
                                                    const StepCoef &, const LaunchCfg &);
}  // namespace lbm
