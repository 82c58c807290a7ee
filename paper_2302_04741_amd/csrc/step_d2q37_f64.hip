// Fused step kernels for D2Q37 with double storage (all equilibrium and force orders),
// and the access-pattern diagnostic.
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_step_ls<0, double>(int, int, const void *, void *, const GridDims &,
                                               const ForceDesc &, const StepCoef &,
                                               const LaunchCfg &);
template hipError_t launch_pattern_ls<0, double>(const void *, void *, const GridDims &,
                                                  const LaunchCfg &);
}  // namespace lbm
