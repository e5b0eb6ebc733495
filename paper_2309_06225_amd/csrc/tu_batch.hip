// Batched pointwise kernel of libgrf for one stage mode
// (compiled once per mode with -DGRF_TU_MODE=1, 2 or 4).
#include "kernels_batch.h"
#include "launch.h"

namespace grf {

template <>
hipError_t launch_point_batch_m<GRF_TU_MODE>(int sa, int grid, const BatchBoxDev* boxes, const CellEntry* cells,
                                             int ncells, int stage, const grf_point_params& pp,
                                             unsigned* status, hipStream_t st) {
  if (sa)
    hipLaunchKernelGGL((k_point_batch<GRF_TU_MODE, 1>), dim3(grid), dim3(kStagedThreads), 0, st, boxes, cells, ncells,
                       stage, pp, status);
  else
    hipLaunchKernelGGL((k_point_batch<GRF_TU_MODE, 0>), dim3(grid), dim3(kStagedThreads), 0, st, boxes, cells, ncells,
                       stage, pp, status);
  return hipGetLastError();
}

// one workgroup per entry
template <>
int grid_point_batch_m<GRF_TU_MODE>(int sa, int64_t work) {
  (void)sa;
  return (int)(work < 1 ? 1 : work);
}

}  // namespace grf
