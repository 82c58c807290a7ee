// Step of a grid between plates (one launch per step) for D2Q37 storage f32 (all equilibrium and force orders).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_wall_step_ls<0, float>(int, int, const void *, void *, const GridDims &,
                                               const ForceDesc &, const StepCoef &,
                                               const LaunchCfg &);
}  // namespace lbm
