// Pointwise right-hand side + RK4 stage with staged inputs, for one stage mode
// (compiled once per mode with -DGRF_TU_MODE=0, 1, 2 or 4), with and without
// shift advection, full theory and decoupling limit.
#include "kernels_staged.h"
#include "launch.h"

namespace grf {

template <>
hipError_t launch_staged_m<GRF_TU_MODE>(int sa, const BoxDev& bd, const grf_point_params& pp, const double* us,
                                        const double* D, const double* u0, double* out, double* acc,
                                        const StageCoef& sc, unsigned* status, hipStream_t st) {
  // sa: bit 0 shift advection, bit 1 the decoupling limit
  const int64_t nblk = (bd.ncell + kStagedThreads - 1) / kStagedThreads;
  const dim3 grid((unsigned)nblk), block(kStagedThreads);
  switch (sa) {
    case 1:
      hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, 1>), grid, block, 0, st, bd, pp, us, D, u0, out, acc, sc, status);
      break;
    case 2:
      hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, 0, true>), grid, block, 0, st, bd, pp, us, D, u0, out, acc, sc,
                         status);
      break;
    case 3:
      hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, 1, true>), grid, block, 0, st, bd, pp, us, D, u0, out, acc, sc,
                         status);
      break;
    default:
      hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, 0>), grid, block, 0, st, bd, pp, us, D, u0, out, acc, sc, status);
      break;
  }
  return hipGetLastError();
}

}  // namespace grf
