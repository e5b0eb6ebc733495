// Stencil-stage, ghost-fill, reduction and elementwise kernels of libgrf and
// their host launchers.
#include "kernels_fwd.h"
#include "kernels_batch.h"
#include "kernels_vjp.h"
#include "launch.h"

namespace grf {


// ---------------------------------------------------------------------------
// Periodic ghost fill, one axis per launch (x, then y over x-ghosts, then z over
// everything), so that edges and corners end up congruent to interior cells.
__global__ void k_periodic(BoxDev b, double* __restrict__ u, int axis) {
  const int n[3] = {b.nx, b.ny, b.nz};
  const int g = b.ng;
  // extents of the ghost slab of this axis in state coordinates
  int ext[3], off[3];
  for (int d = 0; d < 3; ++d) {
    if (d == axis) {
      ext[d] = 2 * g;
      off[d] = 0;
    } else if (d < axis) {
      ext[d] = n[d] + 2 * g;
      off[d] = 0;
    } else {
      ext[d] = n[d];
      off[d] = g;
    }
  }
  const int64_t total = (int64_t)ext[0] * ext[1] * ext[2];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total * NF) return;
  const int f = (int)(e / total);
  int64_t r = e % total;
  int x[3];
  x[0] = (int)(r % ext[0]);
  r /= ext[0];
  x[1] = (int)(r % ext[1]);
  x[2] = (int)(r / ext[1]);
  int src[3];
  for (int d = 0; d < 3; ++d) {
    int v = x[d] + off[d];
    if (d == axis) {
      const int q = x[d];                 // 0 .. 2g-1
      v = q < g ? q : n[d] + q;           // ghost state coordinate
      src[d] = (((v - g) % n[d]) + n[d]) % n[d] + g;  // congruent interior cell
      x[d] = v;
    } else {
      x[d] = v;
      src[d] = v;
    }
  }
  const int64_t base = (int64_t)f * b.fs;
  u[base + (int64_t)x[2] * b.sz + (int64_t)x[1] * b.sy + x[0]] =
      u[base + (int64_t)src[2] * b.sz + (int64_t)src[1] * b.sy + src[0]];
}

// Post-stage algebraic enforcement on interior cells, in place:
// h <- h det(h)^(-1/3); A <- A - 1/3 h tr_h(A) with the corrected h;
// chi <- max(chi, chi_min); lapse <- max(lapse, lapse_min).
__global__ void k_enforce(BoxDev b, double* __restrict__ u, double chi_min, double lapse_min) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.ncell) return;
  const int i = (int)(c % b.nx);
  const int64_t r = c / b.nx;
  const int j = (int)(r % b.ny);
  const int k = (int)(r / b.ny);
  const int64_t s = (int64_t)(k + 3) * b.sz + (int64_t)(j + 3) * b.sy + (i + 3);
  double h[6], A[6];
  for (int q = 0; q < 6; ++q) {
    h[q] = u[(int64_t)(1 + q) * b.fs + s];
    A[q] = u[(int64_t)(8 + q) * b.fs + s];
  }
  // packed order xx, xy, xz, yy, yz, zz
  const double det = h[0] * (h[3] * h[5] - h[4] * h[4]) - h[1] * (h[1] * h[5] - h[4] * h[2]) +
                     h[2] * (h[1] * h[4] - h[3] * h[2]);
  const double f = 1.0 / cbrt(det);
  for (int q = 0; q < 6; ++q) h[q] *= f;
  const double d2 = h[0] * (h[3] * h[5] - h[4] * h[4]) - h[1] * (h[1] * h[5] - h[4] * h[2]) +
                    h[2] * (h[1] * h[4] - h[3] * h[2]);
  const double id = 1.0 / d2;
  const double hu[6] = {(h[3] * h[5] - h[4] * h[4]) * id, (h[2] * h[4] - h[1] * h[5]) * id,
                        (h[1] * h[4] - h[2] * h[3]) * id, (h[0] * h[5] - h[2] * h[2]) * id,
                        (h[1] * h[2] - h[0] * h[4]) * id, (h[0] * h[3] - h[1] * h[1]) * id};
  const double tr = hu[0] * A[0] + hu[3] * A[3] + hu[5] * A[5] + 2.0 * (hu[1] * A[1] + hu[2] * A[2] + hu[4] * A[4]);
  for (int q = 0; q < 6; ++q) {
    u[(int64_t)(1 + q) * b.fs + s] = h[q];
    u[(int64_t)(8 + q) * b.fs + s] = A[q] - h[q] * tr / 3.0;
  }
  const int64_t qc = s, qa = (int64_t)18 * b.fs + s;
  if (u[qc] < chi_min) u[qc] = chi_min;
  if (u[qa] < lapse_min) u[qa] = lapse_min;
}

__global__ void k_status_clear(unsigned* s) {
  if (threadIdx.x == 0) s[threadIdx.x] = 0u;
}

// Fixed-order two-level reduction of the per-cell coupling cotangents.
constexpr int kRedThreads = 256;
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const double* __restrict__ TH, int64_t n,
                                                                int64_t chunk, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  const int q = blockIdx.y;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double s = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += kRedThreads) s += TH[(int64_t)q * n + e];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)q * gridDim.x + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* __restrict__ part, int nparts,
                                                              double* __restrict__ theta_bar) {
  __shared__ double sh[kRedThreads];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int e = threadIdx.x; e < nparts; e += kRedThreads) s += part[(int64_t)q * nparts + e];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) theta_bar[q] += sh[0];
}

// out = a x + b y over n elements (y may be null: out = a x); n counts all
// cells of all fields of a state.
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  out[e] = y ? a * x[e] + b * y[e] : a * x[e];
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = v;
}


// ---------------------------------------------------------------------------
template <int TX, int TY, int TZ>
int tiles_of(const BoxDev& b) {
  return ((b.nx + TX - 1) / TX) * ((b.ny + TY - 1) / TY) * ((b.nz + TZ - 1) / TZ);
}

int tiles_of_variant(int v, const BoxDev& b) {
  switch (v) {
    case 5: return zm_items<16, 8, 32>(b);
    case 6: return zm_items<32, 8, 32>(b);
    case 8: return zm_items<16, 16, 32>(b);
    case 1: return tiles_of<32, 4, 4>(b);
    case 2: return tiles_of<8, 8, 8>(b);
    case 3: return tiles_of<16, 16, 2>(b);
    case 4: return tiles_of<64, 4, 2>(b);
    default: return tiles_of<16, 8, 4>(b);
  }
}

template <int TX, int TY, int TZ>
hipError_t launch_deriv_t(const BoxDev& bd, const double* u, double* D, double sigma, int sa, double* UP,
                          hipStream_t st) {
  hipLaunchKernelGGL((k_deriv<TX, TY, TZ>), dim3(tiles_of<TX, TY, TZ>(bd), NF), dim3(TX * TY * TZ), 0, st, bd, u, D,
                     sigma, sa, UP);
  return hipGetLastError();
}

template <int TX, int TY, int ZC, bool XCDMAP, int ORD = 4, int H = 3>
hipError_t launch_deriv_zm_t(const BoxDev& bd, const double* u, double* D, double sigma, int sa, double* UP,
                             hipStream_t st) {
  const int64_t items = (int64_t)((bd.nx + TX - 1) / TX) * ((bd.ny + TY - 1) / TY) * ((bd.nz + ZC - 1) / ZC) * NF;
  hipLaunchKernelGGL((k_deriv_zm<TX, TY, ZC, XCDMAP, ORD, H>), dim3((unsigned)items), dim3(TX * TY), 0, st, bd, u,
                     D, sigma, sa, UP);
  return hipGetLastError();
}

hipError_t launch_deriv6(const BoxDev& bd, const double* u, double* D, double sigma, int sa, double* UP,
                         hipStream_t st) {
  // the 128x8 column measured slower here (11.9 against 10.1 ms per 128^3 step)
  if (bd.ng == 4) return launch_deriv_zm_t<32, 8, 32, true, 6, 4>(bd, u, D, sigma, sa, UP, st);
  return launch_deriv_zm_t<32, 8, 32, true, 6>(bd, u, D, sigma, sa, UP, st);
}

hipError_t launch_deriv(int variant, const BoxDev& bd, const double* u, double* D, double sigma, int sa, double* UP,
                        hipStream_t st) {
  switch (variant) {
    case 5: return launch_deriv_zm_t<16, 8, 32, true>(bd, u, D, sigma, sa, UP, st);
    case 6: return launch_deriv_zm_t<32, 8, 32, true>(bd, u, D, sigma, sa, UP, st);
    case 7: return launch_deriv_zm_t<32, 4, 32, true>(bd, u, D, sigma, sa, UP, st);
    case 8: return launch_deriv_zm_t<16, 16, 32, true>(bd, u, D, sigma, sa, UP, st);
    case 9: return launch_deriv_zm_t<128, 8, 32, true>(bd, u, D, sigma, sa, UP, st);
    case 1: return launch_deriv_t<32, 4, 4>(bd, u, D, sigma, sa, UP, st);
    case 2: return launch_deriv_t<8, 8, 8>(bd, u, D, sigma, sa, UP, st);
    case 3: return launch_deriv_t<16, 16, 2>(bd, u, D, sigma, sa, UP, st);
    case 4: return launch_deriv_t<64, 4, 2>(bd, u, D, sigma, sa, UP, st);
    default: return launch_deriv_t<16, 8, 4>(bd, u, D, sigma, sa, UP, st);
  }
}

// Grid of the batched stencil stage: one workgroup per (entry, field).  The
// dispatcher hands workgroups to CUs as others finish, heaviest entries first
// (the list's order), which balanced the 96-box workload better than a
// persistent grid of occupancy x CUs workgroups taking entries in turn (22.99
// against 23.62 ms per step).  The kernels keep their grid-stride loop.
int grid_deriv_batch(int variant, int64_t work) {
  (void)variant;
  return (int)std::min<int64_t>(std::max<int64_t>(work, 1), INT32_MAX);
}

template <int TX, int TY, int TZ>
hipError_t launch_deriv_batch_t(int grid, const BatchBoxDev* boxes, const TileEntry* tiles, int ntiles, int stage,
                                double sigma, int sa, hipStream_t st) {
  hipLaunchKernelGGL((k_deriv_batch<TX, TY, TZ>), dim3(grid), dim3(TX * TY * TZ), 0, st, boxes, tiles, ntiles, stage,
                     sigma, sa);
  return hipGetLastError();
}

hipError_t launch_deriv_batch(int variant, int grid, const BatchBoxDev* boxes, const TileEntry* tiles, int ntiles,
                              int stage, double sigma, int sa, hipStream_t st) {
  switch (variant) {
    case 5:
      hipLaunchKernelGGL((k_deriv_batch_zm<16, 8, 32>), dim3(grid), dim3(128), 0, st, boxes, tiles, ntiles, stage,
                         sigma, sa);
      return hipGetLastError();
    case 6:
      hipLaunchKernelGGL((k_deriv_batch_zm<32, 8, 32>), dim3(grid), dim3(256), 0, st, boxes, tiles, ntiles, stage,
                         sigma, sa);
      return hipGetLastError();
    case 8:
      hipLaunchKernelGGL((k_deriv_batch_zm<16, 16, 32>), dim3(grid), dim3(256), 0, st, boxes, tiles, ntiles, stage,
                         sigma, sa);
      return hipGetLastError();
    case 1: return launch_deriv_batch_t<32, 4, 4>(grid, boxes, tiles, ntiles, stage, sigma, sa, st);
    case 2: return launch_deriv_batch_t<8, 8, 8>(grid, boxes, tiles, ntiles, stage, sigma, sa, st);
    case 3: return launch_deriv_batch_t<16, 16, 2>(grid, boxes, tiles, ntiles, stage, sigma, sa, st);
    case 4: return launch_deriv_batch_t<64, 4, 2>(grid, boxes, tiles, ntiles, stage, sigma, sa, st);
    default: return launch_deriv_batch_t<16, 8, 4>(grid, boxes, tiles, ntiles, stage, sigma, sa, st);
  }
}

hipError_t launch_periodic(const BoxDev& bd, double* u, hipStream_t st) {
  const int n[3] = {bd.nx, bd.ny, bd.nz};
  for (int axis = 0; axis < 3; ++axis) {
    int64_t cells = 2 * bd.ng;
    for (int d = 0; d < 3; ++d)
      if (d != axis) cells *= (d < axis) ? (n[d] + 2 * bd.ng) : n[d];
    const int64_t total = cells * NF;
    hipLaunchKernelGGL(k_periodic, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, bd, u, axis);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_enforce(const BoxDev& bd, double* u, double chi_min, double lapse_min, hipStream_t st) {
  hipLaunchKernelGGL(k_enforce, dim3((unsigned)((bd.ncell + 255) / 256)), dim3(256), 0, st, bd, u, chi_min,
                     lapse_min);
  return hipGetLastError();
}

// Peak probes.  k_fma_peak: every thread runs 8 independent dependent chains of
// FP64 fused multiply-adds (16 flops per chain step); the sum is stored so that
// nothing is removed.  k_copy_peak: a grid-stride copy of n doubles.
__global__ __launch_bounds__(256) void k_fma_peak(int iters, double a, double b, double* __restrict__ out) {
  double v[kPeakChains];
#pragma unroll
  for (int q = 0; q < kPeakChains; ++q) v[q] = (double)(threadIdx.x + q);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kPeakChains; ++q) v[q] = fma(v[q], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kPeakChains; ++q) s += v[q];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_copy_peak(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = x[e];
}

hipError_t launch_fma_peak(int blocks, int iters, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fma_peak, dim3(blocks), dim3(256), 0, st, iters, 1.0 - 1e-9, 1e-9, out);
  return hipGetLastError();
}

hipError_t launch_copy_peak(int blocks, int64_t n, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_peak, dim3(blocks), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}

hipError_t launch_status_clear(unsigned* s, hipStream_t st) {
  hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_vjp_transpose(const BoxDev& bd, const double* u, const double* w, const double* Dbar, double sigma,
                                int sa, int order, double* ubar, hipStream_t st) {
  const int e = 2 * bd.ng;
  const int64_t n = (int64_t)(bd.nx + e) * (bd.ny + e) * (bd.nz + e);
  const dim3 grid((unsigned)((n + kGatherThreads - 1) / kGatherThreads), NF);
  if (bd.ng == 4)
    hipLaunchKernelGGL((k_vjp_gather<kGatherThreads, 6, 4>), grid, dim3(kGatherThreads), 0, st, bd, u, w, Dbar, sigma,
                       sa, ubar);
  else if (order == 6)
    hipLaunchKernelGGL((k_vjp_gather<kGatherThreads, 6>), grid, dim3(kGatherThreads), 0, st, bd, u, w, Dbar, sigma, sa,
                       ubar);
  else
    hipLaunchKernelGGL((k_vjp_gather<kGatherThreads, 4>), grid, dim3(kGatherThreads), 0, st, bd, u, w, Dbar, sigma, sa,
                       ubar);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* TH, int64_t n, int64_t chunk, int nparts, double* part, double* theta_bar,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(nparts, NTH), dim3(kRedThreads), 0, st, TH, n, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(NTH), dim3(kRedThreads), 0, st, part, nparts, theta_bar);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y, out);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v, out);
  return hipGetLastError();
}

}  // namespace grf
