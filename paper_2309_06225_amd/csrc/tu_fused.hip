// Fused stage kernel of libgrf for one stage mode (compiled once per mode with
// -DGRF_TU_MODE=0, 1, 2 or 4).
#include "kernels_fwd.h"
#include "launch.h"

namespace grf {

template <>
hipError_t launch_fused_m<GRF_TU_MODE>(int sa, int grid, const BoxDev& bd, const grf_point_params& pp,
                                       const double* us, const double* u0, double* out, double* acc,
                                       const StageCoef& sc, double* Dwg, double sigma, unsigned* status,
                                       hipStream_t st) {
  if (sa)
    hipLaunchKernelGGL((k_stage_fused<GRF_TU_MODE, 1>), dim3(grid), dim3(kFusedNT), 0, st, bd, pp, us, u0, out, acc, sc,
                       Dwg, sigma, status);
  else
    hipLaunchKernelGGL((k_stage_fused<GRF_TU_MODE, 0>), dim3(grid), dim3(kFusedNT), 0, st, bd, pp, us, u0, out, acc, sc,
                       Dwg, sigma, status);
  return hipGetLastError();
}

template <>
int fused_blocks_per_cu_m<GRF_TU_MODE>(int sa) {
  int per = 1;
  hipError_t e = sa ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stage_fused<GRF_TU_MODE, 1>, kFusedNT, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_stage_fused<GRF_TU_MODE, 0>, kFusedNT, 0);
  return (e == hipSuccess && per > 0) ? per : 1;
}

}  // namespace grf
