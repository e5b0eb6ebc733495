// Pointwise right-hand side + RK4 stage kernel of libgrf for one stage mode
// (compiled once per mode with -DGRF_TU_MODE=0, 1, 2 or 4).
#include "kernels_fwd.h"
#include "launch.h"

namespace grf {

template <>
hipError_t launch_point_m<GRF_TU_MODE>(int sa, const BoxDev& bd, const grf_point_params& pp, const double* us,
                                       const double* D, const double* u0, double* out, double* acc,
                                       const StageCoef& sc, unsigned* status, hipStream_t st) {
  const int64_t nblk = (bd.ncell + kPointThreads - 1) / kPointThreads;
  if (sa)
    hipLaunchKernelGGL((k_point<GRF_TU_MODE, 1>), dim3((unsigned)nblk), dim3(kPointThreads), 0, st, bd, pp, us, D, u0,
                       out, acc, sc, status);
  else
    hipLaunchKernelGGL((k_point<GRF_TU_MODE, 0>), dim3((unsigned)nblk), dim3(kPointThreads), 0, st, bd, pp, us, D, u0,
                       out, acc, sc, status);
  return hipGetLastError();
}

}  // namespace grf
