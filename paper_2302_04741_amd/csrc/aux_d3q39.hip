// Totals and plate kernels for D3Q39.
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_totals_l<1>(int, const void *, double *, double *, const GridDims &,
                                         const StepCoef &, hipStream_t);
template hipError_t launch_wall_setup_l<1>(int, const double *, const double *, int64_t,
                                             double *, hipStream_t);
template hipError_t launch_wall_mass_l<1>(int, const void *, const GridDims &, const StepCoef &,
                                            const LaunchCfg &);
}  // namespace lbm
