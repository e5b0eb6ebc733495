// Pointwise right-hand side + RK4 stage with staged inputs, for one stage mode
// (compiled once per mode with -DGRF_TU_MODE=0, 1, 2 or 4).
#include "kernels_staged.h"
#include "launch.h"

namespace grf {

template <>
hipError_t launch_staged_m<GRF_TU_MODE>(int sa, const BoxDev& bd, const grf_point_params& pp, const double* us,
                                        const double* D, const double* u0, double* out, double* acc,
                                        const StageCoef& sc, unsigned* status, hipStream_t st) {
  const int64_t nblk = (bd.ncell + kStagedThreads - 1) / kStagedThreads;
  if (sa)
    hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, 1>), dim3((unsigned)nblk), dim3(kStagedThreads), 0, st, bd, pp,
                       us, D, u0, out, acc, sc, status);
  else
    hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, 0>), dim3((unsigned)nblk), dim3(kStagedThreads), 0, st, bd, pp,
                       us, D, u0, out, acc, sc, status);
  return hipGetLastError();
}

}  // namespace grf
