// Diagnostics per interior cell from the derivative record of the stencil
// stage and the state: the Hamiltonian and momentum constraints (WHICH = 0)
// the energy densities of the canonical, X^2 and Gauss-Bonnet terms of the
// action (WHICH = 1), and the Gauss-Bonnet invariant with the weak-coupling
// indicators (WHICH = 2); WHICH = 3: the constraints in the decoupling limit
// (no scalar sources).
#include "kernels_fwd.h"
#include "launch.h"

namespace grf {

template <int WHICH>
__global__ __launch_bounds__(kPointThreads) void k_constraints(BoxDev b, grf_point_params P,
                                                               const double* __restrict__ us,
                                                               const double* __restrict__ D,
                                                               double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.ncell) return;
  const int i = (int)(c % b.nx);
  const int64_t r = c / b.nx;
  const int j = (int)(r % b.ny);
  const int k = (int)(r / b.ny);
  const int64_t s = (int64_t)(k + 3) * b.sz + (int64_t)(j + 3) * b.sy + (i + 3);
#define GRF_U(f) us[(int64_t)(f) * b.fs + s]
#define GRF_D(cc) D[(int64_t)(cc) * b.ncell + c]
#define GRF_P(n) P.n
#define GRF_CON(q, v) out[(int64_t)(q) * b.ncell + c] = (v)
  if constexpr (WHICH == 0) {
#include "gen/gen_constraints.inc"
  } else if constexpr (WHICH == 3) {
#include "gen/gen_constraints_dec.inc"
  } else if constexpr (WHICH == 1) {
#include "gen/gen_energy.inc"
  } else {
#include "gen/gen_coupling.inc"
  }
#undef GRF_CON
#undef GRF_P
#undef GRF_D
#undef GRF_U
}

hipError_t launch_constraints(int which, const BoxDev& bd, const grf_point_params& pp, const double* u,
                              const double* D, double* out, hipStream_t st) {
  const int64_t nblk = (bd.ncell + kPointThreads - 1) / kPointThreads;
  if (which == 0)
    hipLaunchKernelGGL(k_constraints<0>, dim3((unsigned)nblk), dim3(kPointThreads), 0, st, bd, pp, u, D, out);
  else if (which == 3)
    hipLaunchKernelGGL(k_constraints<3>, dim3((unsigned)nblk), dim3(kPointThreads), 0, st, bd, pp, u, D, out);
  else if (which == 1)
    hipLaunchKernelGGL(k_constraints<1>, dim3((unsigned)nblk), dim3(kPointThreads), 0, st, bd, pp, u, D, out);
  else
    hipLaunchKernelGGL(k_constraints<2>, dim3((unsigned)nblk), dim3(kPointThreads), 0, st, bd, pp, u, D, out);
  return hipGetLastError();
}

}  // namespace grf
