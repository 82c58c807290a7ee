// Initialisation, moments, heat-flux, totals and plate kernels for D3Q39.
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_init_l<1>(int, int, int, const double *, const double *,
                                       const double *, void *, const GridDims &,
                                       const ForceDesc &, const StepCoef &, const LaunchCfg &);
template hipError_t launch_moments_l<1>(int, const void *, double *, double *, double *,
                                          const GridDims &, const ForceDesc &, const StepCoef &,
                                          const LaunchCfg &);
template hipError_t launch_heat_flux_l<1>(int, int, int, const void *, double *,
                                            const GridDims &, const ForceDesc &,
                                            const StepCoef &, const LaunchCfg &);
template hipError_t launch_totals_l<1>(int, const void *, double *, double *, const GridDims &,
                                         const StepCoef &, hipStream_t);
template hipError_t launch_wall_setup_l<1>(int, const double *, const double *, int64_t,
                                             double *, hipStream_t);
template hipError_t launch_wall_mass_l<1>(int, const void *, const GridDims &, const StepCoef &,
                                            const LaunchCfg &);
}  // namespace lbm
