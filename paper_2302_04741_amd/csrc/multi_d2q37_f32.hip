// Multi-grid (batched) step kernels for D2Q37 storage f32 (all equilibrium and force orders).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_multi_step_ls<0, float>(int, int, const BatchLaunch &);
}  // namespace lbm
