// Host-side launchers of libgrf's kernels.  Each is defined in the translation
// unit that instantiates its kernel (so the large pointwise kernels compile in
// parallel); the C-ABI entry points in libgrf.hip call them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/grf.h"
#include "gen/gen_layout.h"

namespace grf {

struct BoxDev;
struct StageCoef;
struct BatchBoxDev;
struct TileEntry;
struct CellEntry;

constexpr int kTileVariants = 5;      // tiled stencil shapes (single-box and batched calls)
constexpr int kDerivVariants = 10;    // plus z-marching shapes 5..9 (single-box calls)

// stencil stage (variant 0..9), optionally storing the upwinded derivatives
hipError_t launch_deriv(int variant, const BoxDev& bd, const double* u, double* D, double sigma, int sa, double* UP,
                        hipStream_t st);
int tiles_of_variant(int variant, const BoxDev& bd);
// sixth-order stencil stage (the z-marching 32x8x32 form; no upwinded-derivative output)
hipError_t launch_deriv6(const BoxDev& bd, const double* u, double* D, double sigma, int sa, double* UP,
                         hipStream_t st);
// batched stencil stage: tiled variants 0..4 and the z-marching variant 8
hipError_t launch_deriv_batch(int variant, int grid, const BatchBoxDev* boxes, const TileEntry* tiles, int ntiles,
                              int stage, double sigma, int sa, hipStream_t st);
int grid_deriv_batch(int variant, int64_t work);
hipError_t launch_periodic(const BoxDev& bd, double* u, hipStream_t st);
hipError_t launch_status_clear(unsigned* s, hipStream_t st);
// Hamiltonian and momentum constraints of every interior cell (out: [4][ncell])
// which: 0 Hamiltonian and momentum constraints (4 outputs), 1 energy densities (3 outputs),
// 2 Gauss-Bonnet invariant and weak-coupling indicators (3 outputs)
hipError_t launch_constraints(int which, const BoxDev& bd, const grf_point_params& pp, const double* u,
                              const double* D, double* out, hipStream_t st);
constexpr int kPeakChains = 8;  // independent FMA chains per thread of the FP64 peak probe
hipError_t launch_fma_peak(int blocks, int iters, double* out, hipStream_t st);
hipError_t launch_copy_peak(int blocks, int64_t n, const double* x, double* y, hipStream_t st);
hipError_t launch_enforce(const BoxDev& bd, double* u, double chi_min, double lapse_min, hipStream_t st);

// per-face boundary rules, device form of grf_bc (sign: reflection parity per axis and field)
struct BcDev {
  int rule[6];
  int extrap_order;
  double origin[3], centre[3], h[3], i2h[3];
  double speed[GRF_NFIELDS], asymptote[GRF_NFIELDS];
  double sign[3][GRF_NFIELDS];
};
int64_t ghost_cells(const BoxDev& bd);
// refill of the periodic, reflective and extrapolating ghosts (z, y, x)
hipError_t launch_bc_fill(const BoxDev& bd, const BcDev& bc, double* u, hipStream_t st);
// mode 0: radiative right-hand side into the ghosts of out (0 off Sommerfeld faces);
// 1, 2, 4: RK4 stage update of the Sommerfeld ghosts of out
hipError_t launch_bc_ghost(int mode, const BoxDev& bd, const BcDev& bc, const double* us, const double* u0,
                           double* out, double* gacc, const StageCoef& sc, hipStream_t st);

// pointwise right-hand side + stage update (mode 0, 1, 2, 4)
template <int MODE>
hipError_t launch_point_m(int sa, const BoxDev& bd, const grf_point_params& pp, const double* us, const double* D,
                          const double* u0, double* out, double* acc, const StageCoef& sc, unsigned* status,
                          hipStream_t st);
template <> hipError_t launch_point_m<0>(int, const BoxDev&, const grf_point_params&, const double*, const double*,
                                         const double*, double*, double*, const StageCoef&, unsigned*, hipStream_t);
template <> hipError_t launch_point_m<1>(int, const BoxDev&, const grf_point_params&, const double*, const double*,
                                         const double*, double*, double*, const StageCoef&, unsigned*, hipStream_t);
template <> hipError_t launch_point_m<2>(int, const BoxDev&, const grf_point_params&, const double*, const double*,
                                         const double*, double*, double*, const StageCoef&, unsigned*, hipStream_t);
template <> hipError_t launch_point_m<4>(int, const BoxDev&, const grf_point_params&, const double*, const double*,
                                         const double*, double*, double*, const StageCoef&, unsigned*, hipStream_t);

// batched pointwise stage (stage 1 -> mode 1, stages 2-3 -> mode 2, stage 4 -> mode 4)
template <int MODE>
hipError_t launch_point_batch_m(int sa, int grid, const BatchBoxDev* boxes, const CellEntry* cells, int ncells,
                                int stage, const grf_point_params& pp, unsigned* status, hipStream_t st);
template <> hipError_t launch_point_batch_m<1>(int, int, const BatchBoxDev*, const CellEntry*, int, int,
                                               const grf_point_params&, unsigned*, hipStream_t);
template <> hipError_t launch_point_batch_m<2>(int, int, const BatchBoxDev*, const CellEntry*, int, int,
                                               const grf_point_params&, unsigned*, hipStream_t);
template <> hipError_t launch_point_batch_m<4>(int, int, const BatchBoxDev*, const CellEntry*, int, int,
                                               const grf_point_params&, unsigned*, hipStream_t);
template <int MODE>
int grid_point_batch_m(int sa, int64_t work);
template <> int grid_point_batch_m<1>(int, int64_t);
template <> int grid_point_batch_m<2>(int, int64_t);
template <> int grid_point_batch_m<4>(int, int64_t);

// pointwise right-hand side + stage update with inputs staged through LDS (same
// arguments and results as launch_point_m)
template <int MODE>
hipError_t launch_staged_m(int sa, const BoxDev& bd, const grf_point_params& pp, const double* us, const double* D,
                           const double* u0, double* out, double* acc, const StageCoef& sc, unsigned* status,
                           hipStream_t st);
#define GRF_DECL_STAGED(M)                                                                                      \
  template <> hipError_t launch_staged_m<M>(int, const BoxDev&, const grf_point_params&, const double*,        \
                                            const double*, const double*, double*, double*, const StageCoef&, \
                                            unsigned*, hipStream_t);
GRF_DECL_STAGED(0)
GRF_DECL_STAGED(1)
GRF_DECL_STAGED(2)
GRF_DECL_STAGED(4)
#undef GRF_DECL_STAGED

// VJP pieces
hipError_t launch_vjp_point(int sa, const BoxDev& bd, const grf_point_params& pp, const double* u, const double* D,
                            const double* UP, const double* w, double* ubar, double* Dbar, double* TH,
                            hipStream_t st);
// the same in the decoupling limit
hipError_t launch_vjp_point_dec(int sa, const BoxDev& bd, const grf_point_params& pp, const double* u, const double* D,
                            const double* UP, const double* w, double* ubar, double* Dbar, double* TH,
                            hipStream_t st);
hipError_t launch_vjp_transpose(const BoxDev& bd, const double* u, const double* w, const double* Dbar, double sigma,
                                int sa, int order, double* ubar, hipStream_t st);
hipError_t launch_reduce(const double* TH, int64_t n, int64_t chunk, int nparts, double* part, double* theta_bar,
                         hipStream_t st);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                        hipStream_t st);
hipError_t launch_fill(int64_t n, double v, double* out, hipStream_t st);


}  // namespace grf
