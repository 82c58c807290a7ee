// Resident multi-step kernel for small grids, D2Q37 storage f16 (all equilibrium and force
// orders, with and without plates).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_resident_ls<0, __half>(int, int, void *, void *, const GridDims &,
                                              const ForceDesc &, const StepCoef &,
                                              const LaunchCfg &, int);
}  // namespace lbm
