// Reverse-mode pointwise kernel of libgrf.
#include "kernels_vjp.h"
#include "launch.h"

namespace grf {

hipError_t launch_vjp_point(int sa, const BoxDev& bd, const grf_point_params& pp, const double* u, const double* D,
                            const double* UP, const double* w, double* ubar, double* Dbar, double* TH,
                            hipStream_t st) {
  const unsigned nblk = (unsigned)((bd.ncell + 63) / 64);
  if (sa)
    hipLaunchKernelGGL((k_vjp_point<1>), dim3(nblk), dim3(64), 0, st, bd, pp, u, D, UP, w, ubar, Dbar, TH);
  else
    hipLaunchKernelGGL((k_vjp_point<0>), dim3(nblk), dim3(64), 0, st, bd, pp, u, D, UP, w, ubar, Dbar, TH);
  return hipGetLastError();
}

}  // namespace grf
