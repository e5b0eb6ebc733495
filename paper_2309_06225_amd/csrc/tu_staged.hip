// Pointwise right-hand side + RK4 stage with staged inputs, for one stage mode
// (compiled once per mode with -DGRF_TU_MODE=0, 1, 2 or 4), with and without
// shift advection, full theory, decoupling limit and full theory with the
// general coupling.
#include "kernels_staged.h"
#include "launch.h"

namespace grf {

template <>
hipError_t launch_staged_m<GRF_TU_MODE>(int sa, const BoxDev& bd, const grf_point_params& pp, const double* us,
                                        const double* D, const double* u0, double* out, double* acc,
                                        const StageCoef& sc, unsigned* status, hipStream_t st) {
  // sa: bit 0 shift advection; bits 1-2 the variant (0 full theory, 1 the
  // decoupling limit, 2 the full theory with the general coupling)
  const int64_t nblk = (bd.ncell + kStagedThreads - 1) / kStagedThreads;
  const dim3 grid((unsigned)nblk), block(kStagedThreads);
#define GRF_LAUNCH_STAGED(S, V) \
  hipLaunchKernelGGL((k_point_staged<GRF_TU_MODE, S, V>), grid, block, 0, st, bd, pp, us, D, u0, out, acc, sc, status)
  switch (sa) {
    case 1: GRF_LAUNCH_STAGED(1, 0); break;
    case 2: GRF_LAUNCH_STAGED(0, 1); break;
    case 3: GRF_LAUNCH_STAGED(1, 1); break;
    case 4: GRF_LAUNCH_STAGED(0, 2); break;
    case 5: GRF_LAUNCH_STAGED(1, 2); break;
    default: GRF_LAUNCH_STAGED(0, 0); break;
  }
#undef GRF_LAUNCH_STAGED
  return hipGetLastError();
}

}  // namespace grf
