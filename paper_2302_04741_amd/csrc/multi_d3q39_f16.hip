// Multi-grid (batched) step kernels for D3Q39 storage f16 (all equilibrium and force orders).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_multi_step_ls<1, __half>(int, int, const BatchLaunch &);
}  // namespace lbm
