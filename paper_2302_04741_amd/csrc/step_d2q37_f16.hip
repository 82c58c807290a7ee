// Fused step kernels for D2Q37 with F16 deviation storage (FP32 arithmetic).
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_step_ls<0, __half>(int, int, const void *, void *, const GridDims &,
                                                const ForceDesc &, const StepCoef &,
                                                const LaunchCfg &);
}  // namespace lbm
