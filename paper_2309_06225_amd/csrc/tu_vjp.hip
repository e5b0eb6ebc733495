// Reverse-mode pointwise kernel of libgrf, for the full theory or (compiled
// with -DGRF_VJP_DEC=1, in a translation unit of its own) the decoupling limit.
#include "kernels_vjp.h"
#include "launch.h"

#ifndef GRF_VJP_DEC
#define GRF_VJP_DEC 0
#endif

namespace grf {

#if GRF_VJP_DEC
hipError_t launch_vjp_point_dec(int sa, const BoxDev& bd, const grf_point_params& pp, const double* u,
                                const double* D, const double* UP, const double* w, double* ubar, double* Dbar,
                                double* TH, hipStream_t st) {
#else
hipError_t launch_vjp_point(int sa, const BoxDev& bd, const grf_point_params& pp, const double* u, const double* D,
                            const double* UP, const double* w, double* ubar, double* Dbar, double* TH,
                            hipStream_t st) {
#endif
  const unsigned nblk = (unsigned)((bd.ncell + 63) / 64);
  if (sa)
    hipLaunchKernelGGL((k_vjp_point<1, GRF_VJP_DEC>), dim3(nblk), dim3(64), 0, st, bd, pp, u, D, UP, w, ubar, Dbar,
                       TH);
  else
    hipLaunchKernelGGL((k_vjp_point<0, GRF_VJP_DEC>), dim3(nblk), dim3(64), 0, st, bd, pp, u, D, UP, w, ubar, Dbar,
                       TH);
  return hipGetLastError();
}

}  // namespace grf
