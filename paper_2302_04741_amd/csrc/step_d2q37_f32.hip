// Fused step kernels for D2Q37 with float storage (all equilibrium and force orders).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_step_ls<0, float>(int, int, const void *, void *, const GridDims &,
                                               const ForceDesc &, const StepCoef &,
                                               const LaunchCfg &);
}  // namespace lbm
