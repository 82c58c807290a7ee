// Resident multi-step kernel for small grids, D3Q39 storage f64 (all equilibrium and force
// orders, with and without plates).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_resident_ls<1, double>(int, int, void *, void *, const GridDims &,
                                              const ForceDesc &, const StepCoef &,
                                              const LaunchCfg &, int);
}  // namespace lbm
