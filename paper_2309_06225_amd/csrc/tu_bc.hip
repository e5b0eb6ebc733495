// Per-face boundary rules (Key features, "Boundary Conditions": periodic,
// reflective, extrapolating and Sommerfeld faces) and their host launchers.
//
// Ownership: every ghost cell belongs to one face, the x face when its x index
// lies outside the interior, else the y face when its y index does, else the z
// face.  Frozen and Sommerfeld ghosts are integrated by the RK4 stage (right-
// hand side 0 and the radiative one); periodic, reflective and extrapolating
// ghosts are refilled from the new stage state, z faces first, then y, then
// x, so that every face reads only cells that are already final.
#include "kernels_fwd.h"
#include "launch.h"

namespace grf {

// each product rounded on its own, as in the stage update of the interior
#pragma clang fp contract(off)

// Ghost region of one axis's two faces in state coordinates (cell offsets from
// the first ghost): the axis itself spans its 2 ng ghost layers; lower axes
// (which own their own ghosts) span only the interior, higher axes span
// everything.
struct Slab {
  int ext[3];  // extents along x, y, z
  int off[3];  // first coordinate (0 = outermost ghost, ng = first interior cell)
  __host__ __device__ int64_t count() const { return (int64_t)ext[0] * ext[1] * ext[2]; }
};

__host__ __device__ inline Slab slab_of(const BoxDev& b, int axis) {
  const int n[3] = {b.nx, b.ny, b.nz};
  const int g = b.ng;
  Slab s;
  for (int d = 0; d < 3; ++d) {
    if (d == axis) {
      s.ext[d] = 2 * g;
      s.off[d] = 0;
    } else if (d < axis) {
      s.ext[d] = n[d];
      s.off[d] = g;
    } else {
      s.ext[d] = n[d] + 2 * g;
      s.off[d] = 0;
    }
  }
  return s;
}

// state coordinates (0 .. n+2ng-1) of element e of the slab; the axis's ghost
// layers 0..2ng-1 map to 0..ng-1 (low face) and n+ng..n+2ng-1 (high face)
__device__ __forceinline__ void slab_cell(const BoxDev& b, const Slab& s, int axis, int64_t e, int x[3]) {
  const int n[3] = {b.nx, b.ny, b.nz};
  int64_t r = e;
  for (int d = 0; d < 3; ++d) {
    const int v = (int)(r % s.ext[d]);
    r /= s.ext[d];
    x[d] = s.off[d] + v;
    if (d == axis && v >= b.ng) x[d] = n[d] + v;  // ng .. 2ng-1 -> n+ng .. n+2ng-1
  }
}

__device__ __forceinline__ int64_t state_at(const BoxDev& b, const int x[3]) {
  return (int64_t)x[2] * b.sz + (int64_t)x[1] * b.sy + x[0];
}

// One axis of the refill: every ghost of this axis's faces whose rule is
// periodic, reflective or extrapolating takes its value from cells interior
// along the axis.
__global__ __launch_bounds__(256) void k_bc_fill(BoxDev b, BcDev bc, int axis, double* __restrict__ u) {
  const Slab s = slab_of(b, axis);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s.count()) return;
  int x[3];
  slab_cell(b, s, axis, e, x);
  const int n = axis == 0 ? b.nx : axis == 1 ? b.ny : b.nz;
  const int m = x[axis] - b.ng;  // interior index along the axis (negative on the low face)
  const bool low = m < 0;
  const int rule = bc.rule[2 * axis + (low ? 0 : 1)];
  if (rule != GRF_FACE_PERIODIC && rule != GRF_FACE_REFLECTIVE && rule != GRF_FACE_EXTRAPOLATING) return;
  const int64_t dst = state_at(b, x);
  const int64_t step = axis == 0 ? 1 : axis == 1 ? (int64_t)b.sy : b.sz;  // one cell along the axis
  const int64_t base = dst - (int64_t)m * step;                          // interior index 0 along the axis
  if (rule == GRF_FACE_PERIODIC) {
    const int mm = ((m % n) + n) % n;
    const int64_t src = base + (int64_t)mm * step;
    for (int f = 0; f < NF; ++f) u[(int64_t)f * b.fs + dst] = u[(int64_t)f * b.fs + src];
  } else if (rule == GRF_FACE_REFLECTIVE) {
    const int mm = low ? -1 - m : 2 * n - 1 - m;
    const int64_t src = base + (int64_t)mm * step;
    for (int f = 0; f < NF; ++f) u[(int64_t)f * b.fs + dst] = bc.sign[axis][f] * u[(int64_t)f * b.fs + src];
  } else {
    const int edge = low ? 0 : n - 1;
    const int64_t s1 = base + (int64_t)edge * step;
    const int64_t s2 = base + (int64_t)(low ? 1 : n - 2) * step;
    const double dist = (double)(low ? -m : m - edge);
    for (int f = 0; f < NF; ++f) {
      const double ue = u[(int64_t)f * b.fs + s1];
      u[(int64_t)f * b.fs + dst] = bc.extrap_order == 0 ? ue : ue + dist * (ue - u[(int64_t)f * b.fs + s2]);
    }
  }
}

// Radiative right-hand side -v (x^a d_a f + f - f_inf) / r of every field at
// ghost cell x (state coordinates) of a Sommerfeld face, with second-order
// differences, one-sided towards the interior along axes where the cell is a
// ghost and centred along the others; then MODE's use of it (0: store it in
// out, 1/2/4: RK4 stage update with the ghost accumulator gacc).
template <int MODE>
__device__ __forceinline__ void sommerfeld_cell(const BoxDev& b, const BcDev& bc, const int x[3], int64_t g,
                                                int64_t nghost, const double* __restrict__ us,
                                                const double* __restrict__ u0, double* __restrict__ out,
                                                double* __restrict__ gacc, StageCoef sc) {
  const int n[3] = {b.nx, b.ny, b.nz};
  const int64_t step[3] = {1, (int64_t)b.sy, b.sz};
  const int64_t c = state_at(b, x);
  double rel[3];
  double r2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    rel[a] = bc.origin[a] + (double)(x[a] - b.ng) * bc.h[a] - bc.centre[a];
    r2 += rel[a] * rel[a];
  }
  const double inv_r = 1.0 / sqrt(r2);
  // per axis: stencil kind and weights on (c, c + dir step, c + 2 dir step)
  int kind[3];
  for (int a = 0; a < 3; ++a) kind[a] = x[a] < b.ng ? -1 : (x[a] >= n[a] + b.ng ? 1 : 0);
  for (int f = 0; f < NF; ++f) {
    const double* uf = us + (int64_t)f * b.fs;
    const double val = uf[c];
    double xd = 0.0;
    for (int a = 0; a < 3; ++a) {
      double d;
      if (kind[a] == 0) {
        d = (uf[c + step[a]] - uf[c - step[a]]) * bc.i2h[a];
      } else {
        // towards the interior: dir = +1 on a low face, -1 on a high face
        const int64_t s1 = kind[a] < 0 ? step[a] : -step[a];
        const double one_sided = -3.0 * val + 4.0 * uf[c + s1] - uf[c + 2 * s1];
        d = (kind[a] < 0 ? one_sided : -one_sided) * bc.i2h[a];
      }
      xd += rel[a] * d;
    }
    const double k = -bc.speed[f] * (xd + (val - bc.asymptote[f])) * inv_r;
    const int64_t q = (int64_t)f * b.fs + c;
    const int64_t qa = (int64_t)f * nghost + g;
    if constexpr (MODE == 0) {
      out[q] = k;
    } else if constexpr (MODE == 1) {
      gacc[qa] = k;
      out[q] = u0[q] + sc.cnext * k;
    } else if constexpr (MODE == 2) {
      gacc[qa] = gacc[qa] + 2.0 * k;
      out[q] = u0[q] + sc.cnext * k;
    } else {
      out[q] = u0[q] + sc.cnext * (gacc[qa] + k);
    }
  }
}

// Every ghost cell in the order of the three slabs (x, y, z); g is its index in
// the ghost accumulator.  MODE 0 writes the ghost right-hand side (0 on faces
// that are not Sommerfeld); MODE 1/2/4 update the Sommerfeld ghosts only.
template <int MODE>
__global__ __launch_bounds__(256) void k_bc_ghost(BoxDev b, BcDev bc, const double* __restrict__ us,
                                                  const double* __restrict__ u0, double* __restrict__ out,
                                                  double* __restrict__ gacc, StageCoef sc) {
  const Slab s0 = slab_of(b, 0), s1 = slab_of(b, 1), s2 = slab_of(b, 2);
  const int64_t n0 = s0.count(), n1 = s1.count(), n2 = s2.count();
  const int64_t nghost = n0 + n1 + n2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nghost) return;
  int axis;
  int64_t e;
  if (g < n0) {
    axis = 0;
    e = g;
  } else if (g < n0 + n1) {
    axis = 1;
    e = g - n0;
  } else {
    axis = 2;
    e = g - n0 - n1;
  }
  int x[3];
  slab_cell(b, axis == 0 ? s0 : axis == 1 ? s1 : s2, axis, e, x);
  const bool low = x[axis] < b.ng;
  const int rule = bc.rule[2 * axis + (low ? 0 : 1)];
  if (rule == GRF_FACE_SOMMERFELD) {
    sommerfeld_cell<MODE>(b, bc, x, g, nghost, us, u0, out, gacc, sc);
  } else if constexpr (MODE == 0) {
    const int64_t c = state_at(b, x);
    for (int f = 0; f < NF; ++f) out[(int64_t)f * b.fs + c] = 0.0;
  }
}

int64_t ghost_cells(const BoxDev& bd) {
  return slab_of(bd, 0).count() + slab_of(bd, 1).count() + slab_of(bd, 2).count();
}

hipError_t launch_bc_fill(const BoxDev& bd, const BcDev& bc, double* u, hipStream_t st) {
  for (int axis = 2; axis >= 0; --axis) {
    const bool any = bc.rule[2 * axis] != GRF_FACE_FROZEN && bc.rule[2 * axis] != GRF_FACE_SOMMERFELD;
    const bool any2 = bc.rule[2 * axis + 1] != GRF_FACE_FROZEN && bc.rule[2 * axis + 1] != GRF_FACE_SOMMERFELD;
    if (!any && !any2) continue;
    const int64_t total = slab_of(bd, axis).count();
    hipLaunchKernelGGL(k_bc_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, bd, bc, axis, u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_bc_ghost(int mode, const BoxDev& bd, const BcDev& bc, const double* us, const double* u0,
                           double* out, double* gacc, const StageCoef& sc, hipStream_t st) {
  const int64_t total = ghost_cells(bd);
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_bc_ghost<0>, grid, block, 0, st, bd, bc, us, u0, out, gacc, sc); break;
    case 1: hipLaunchKernelGGL(k_bc_ghost<1>, grid, block, 0, st, bd, bc, us, u0, out, gacc, sc); break;
    case 2: hipLaunchKernelGGL(k_bc_ghost<2>, grid, block, 0, st, bd, bc, us, u0, out, gacc, sc); break;
    default: hipLaunchKernelGGL(k_bc_ghost<4>, grid, block, 0, st, bd, bc, us, u0, out, gacc, sc); break;
  }
  return hipGetLastError();
}

}  // namespace grf
