// Initialisation, moments and heat-flux kernels for D3Q39 storage f16 (all orders), and the
// F16 stochastic rounding of plain arrays.
#include "lbm_launch.h"

namespace lbm {
template hipError_t launch_init_ls<1, __half>(int, int, const double *, const double *,
                                               const double *, void *, const GridDims &,
                                               const ForceDesc &, const StepCoef &,
                                               const LaunchCfg &);
template hipError_t launch_moments_ls<1, __half>(const void *, double *, double *, double *,
                                                  const GridDims &, const ForceDesc &,
                                                  const StepCoef &, const LaunchCfg &);
template hipError_t launch_heat_flux_ls<1, __half>(int, int, const void *, double *,
                                                    const GridDims &, const ForceDesc &,
                                                    const StepCoef &, const LaunchCfg &);

// half_sr over plain arrays (grid-stride: any n with a bounded grid)
__global__ void __launch_bounds__(256) round_f16_sr_kernel(const float *__restrict__ v,
                                                           const uint32_t *__restrict__ seed,
                                                           uint16_t *__restrict__ out, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += stride)
        out[k] = __builtin_bit_cast(uint16_t, half_sr(v[k], seed[k]));
}

hipError_t launch_round_f16_sr(const float *v, const uint32_t *seed, uint16_t *out, int64_t n,
                                hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(round_f16_sr_kernel, dim3(uint32_t(blocks)), dim3(256), 0, stream, v, seed,
                       out, n);
    return hipGetLastError();
}
}  // namespace lbm
