// Initialisation, moments and heat-flux kernels for D3Q39 storage f32 (all orders).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_init_ls<1, float>(int, int, const double *, const double *,
                                               const double *, void *, const GridDims &,
                                               const ForceDesc &, const StepCoef &,
                                               const LaunchCfg &);
template hipError_t launch_moments_ls<1, float>(const void *, double *, double *, double *,
                                                  const GridDims &, const ForceDesc &,
                                                  const StepCoef &, const LaunchCfg &);
template hipError_t launch_heat_flux_ls<1, float>(int, int, const void *, double *,
                                                    const GridDims &, const ForceDesc &,
                                                    const StepCoef &, const LaunchCfg &);
}  // namespace lbm
