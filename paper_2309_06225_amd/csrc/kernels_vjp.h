// Reverse-mode kernels of libgrf: vector-Jacobian product of the right-hand side.
//
// Pass 1 (k_deriv with UP): derivative record D and upwinded derivatives UP at u.
// Pass 2 (k_vjp_point): per interior cell, the generated reverse of the pointwise
//   algebra.  Given w (cotangent of the right-hand side) it adds the cotangent of
//   the cell's own field values to u_bar, stores the cotangents of every stencil
//   input (first/second derivatives, advection sums) in Dbar, adds the shift's
//   share of the advection sums (sum_f adv_bar_f * D^up_k u_f) to u_bar, and
//   stores the cell's coupling cotangents in TH.
// Pass 3 (k_vjp_transpose): for every cell of the box, ghosts included, gathers
//   the transposed stencils: sum over interior source cells c of stencil weight
//   times the cotangent stored at c (and the Kreiss-Oliger stencil applied to w).
// Pass 4 (k_reduce_*): fixed-order tree sum of TH into theta_bar.
#pragma once
#include "kernels_fwd.h"

namespace grf {

constexpr int NTH = 2;
// components of the cotangent record Dbar (same numbering as D, without Kreiss-Oliger)
constexpr int NCOMP_BAR = GRF_OFF_KO;

template <int SHIFTADV>
__global__ __launch_bounds__(64) void k_vjp_point(BoxDev b, grf_point_params P, const double* __restrict__ us,
                                                  const double* __restrict__ D, const double* __restrict__ UP,
                                                  const double* __restrict__ w, double* __restrict__ ubar,
                                                  double* __restrict__ Dbar, double* __restrict__ TH) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.ncell) return;
  const int i = (int)(c % b.nx);
  const int64_t r = c / b.nx;
  const int j = (int)(r % b.ny);
  const int k = (int)(r / b.ny);
  const int64_t s = (int64_t)(k + 3) * b.sz + (int64_t)(j + 3) * b.sy + (i + 3);
  const int64_t nc = b.ncell;
  double ub[NF];
#define GRF_U(f) us[(int64_t)(f) * b.fs + s]
#define GRF_D(cc) D[(int64_t)(cc) * nc + c]
#define GRF_P(n) P.n
#define GRF_W(f) w[(int64_t)(f) * b.fs + s]
#define GRF_BAR_U(f, v) ub[f] = (v)
#define GRF_BAR_D(cc, v) Dbar[(int64_t)(cc) * nc + c] = (v)
#define GRF_BAR_TH(q, v) TH[(int64_t)(q) * nc + c] = (v)
#define GRF_SHIFT_ADVEC (SHIFTADV != 0)
#include "gen/gen_vjp.inc"
#undef GRF_SHIFT_ADVEC
#undef GRF_BAR_U
#undef GRF_BAR_D
#undef GRF_BAR_TH
#undef GRF_W
  // the advection sums beta^k D^up_k u_f also depend on the shift value
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double sb = 0.0;
    for (int f = 0; f < NF; ++f) {
      if (!advected(f, SHIFTADV)) continue;
      sb += Dbar[(int64_t)(GRF_OFF_ADV + f) * nc + c] * UP[(int64_t)(3 * f + d) * nc + c];
    }
    ub[F_SHIFT + d] += sb;
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) ubar[(int64_t)f * b.fs + s] += ub[f];
}

// Stage one cotangent component of the source cells of a tile (+3 halo) into
// LDS; cells outside the interior contribute nothing.
template <int LX, int LY, int LZ, int NT>
__device__ __forceinline__ void stage_src(const BoxDev& b, double* t, int tx0, int ty0, int tz0,
                                          const double* __restrict__ comp) {
  for (int e = threadIdx.x; e < LX * LY * LZ; e += NT) {
    const int lx = e % LX;
    const int r = e / LX;
    const int ly = r % LY;
    const int lz = r / LY;
    // interior coordinates of the source cell (state coordinate - 3)
    const int ix = tx0 - 3 + lx - 3, iy = ty0 - 3 + ly - 3, iz = tz0 - 3 + lz - 3;
    double v = 0.0;
    if (ix >= 0 && ix < b.nx && iy >= 0 && iy < b.ny && iz >= 0 && iz < b.nz)
      v = comp[((int64_t)iz * b.ny + iy) * b.nx + ix];
    t[e] = v;
  }
}

// Upwind split of the advection cotangent: S+ = adv_bar * beta_k where beta_k >= 0, else S-.
template <int LX, int LY, int LZ, int NT>
__device__ __forceinline__ void stage_upwind(const BoxDev& b, double* tp, double* tm, int tx0, int ty0, int tz0,
                                             const double* __restrict__ advbar, const double* __restrict__ u,
                                             int d) {
  for (int e = threadIdx.x; e < LX * LY * LZ; e += NT) {
    const int lx = e % LX;
    const int r = e / LX;
    const int ly = r % LY;
    const int lz = r / LY;
    const int ix = tx0 - 3 + lx - 3, iy = ty0 - 3 + ly - 3, iz = tz0 - 3 + lz - 3;
    double vp = 0.0, vm = 0.0;
    if (ix >= 0 && ix < b.nx && iy >= 0 && iy < b.ny && iz >= 0 && iz < b.nz) {
      const double a = advbar[((int64_t)iz * b.ny + iy) * b.nx + ix];
      const double bd =
          u[(int64_t)(F_SHIFT + d) * b.fs + (int64_t)(iz + 3) * b.sz + (int64_t)(iy + 3) * b.sy + (ix + 3)];
      if (bd >= 0.0)
        vp = a * bd;
      else
        vm = a * bd;
    }
    tp[e] = vp;
    tm[e] = vm;
  }
}

// Transposed stencils.  One workgroup = one field of one TX*TY*TZ tile of the
// full box (ghosts included); u_bar[f] += sum of every stencil's transpose.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_vjp_transpose(BoxDev b, const double* __restrict__ u,
                                                              const double* __restrict__ w,
                                                              const double* __restrict__ Dbar, double ko_sigma,
                                                              int shift_adv, double* __restrict__ ubar) {
  constexpr int LX = TX + 6, LY = TY + 6, LZ = TZ + 6, NT = TX * TY * TZ;
  __shared__ double t0[LZ * LY * LX];
  __shared__ double t1[LZ * LY * LX];
  const int f = blockIdx.y;
  const int NX = b.nx + 6, NY = b.ny + 6, NZ = b.nz + 6;  // full box (state coordinates)
  const int ntx = (NX + TX - 1) / TX, nty = (NY + TY - 1) / TY;
  int tile = blockIdx.x;
  const int tx0 = (tile % ntx) * TX;
  tile /= ntx;
  const int ty0 = (tile % nty) * TY;
  const int tz0 = (tile / nty) * TZ;
  const int ix = threadIdx.x % TX, iy = (threadIdx.x / TX) % TY, iz = threadIdx.x / (TX * TY);
  const int X = tx0 + ix, Y = ty0 + iy, Z = tz0 + iz;  // target, state coordinates
  const bool valid = X < NX && Y < NY && Z < NZ;
  const int c0 = ((iz + 3) * LY + (iy + 3)) * LX + (ix + 3);
  const int st[3] = {1, LX, LX * LY};
  const int64_t nc = b.ncell;
  double acc = 0.0;

  const int s1 = grf_d1_slot[f];
  if (s1 >= 0) {
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      stage_src<LX, LY, LZ, NT>(b, t0, tx0, ty0, tz0, Dbar + (int64_t)(GRF_OFF_D1 + 3 * s1 + d) * nc);
      __syncthreads();
      double s = 0.0;
#pragma unroll
      for (int o = -2; o <= 2; ++o)
        if (o != 0) s += w1[o + 2] * t0[c0 - o * st[d]];
      acc += s * b.i12h[d];
    }
  }
  const int s2 = grf_d2_slot[f];
  if (s2 >= 0) {
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
    const double w2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    const int pure[3] = {0, 3, 5};
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      stage_src<LX, LY, LZ, NT>(b, t0, tx0, ty0, tz0, Dbar + (int64_t)(GRF_OFF_D2 + 6 * s2 + pure[d]) * nc);
      __syncthreads();
      double s = 0.0;
#pragma unroll
      for (int o = -2; o <= 2; ++o) s += w2[o + 2] * t0[c0 - o * st[d]];
      acc += s * b.i12h2[d];
    }
    const int pd[3] = {0, 0, 1}, pe[3] = {1, 2, 2}, pq[3] = {1, 2, 4};
    for (int m = 0; m < 3; ++m) {
      __syncthreads();
      stage_src<LX, LY, LZ, NT>(b, t0, tx0, ty0, tz0, Dbar + (int64_t)(GRF_OFF_D2 + 6 * s2 + pq[m]) * nc);
      __syncthreads();
      double s = 0.0;
#pragma unroll
      for (int a = -2; a <= 2; ++a)
#pragma unroll
        for (int bb = -2; bb <= 2; ++bb)
          if (a != 0 && bb != 0) s += (w1[a + 2] * w1[bb + 2]) * t0[c0 - a * st[pd[m]] - bb * st[pe[m]]];
      acc += s * b.i144[m];
    }
  }
  if (advected(f, shift_adv)) {
    // weights of u(c + o e_k) in the lopsided stencils, o = -3..3
    const double wp[7] = {0.0, 0.0, -3.0, -10.0, 18.0, -6.0, 1.0};
    const double wm[7] = {-1.0, 6.0, -18.0, 10.0, 3.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      stage_upwind<LX, LY, LZ, NT>(b, t0, t1, tx0, ty0, tz0, Dbar + (int64_t)(GRF_OFF_ADV + f) * nc, u, d);
      __syncthreads();
      double s = 0.0;
#pragma unroll
      for (int o = -3; o <= 3; ++o) s += wp[o + 3] * t0[c0 - o * st[d]] + wm[o + 3] * t1[c0 - o * st[d]];
      acc += s * b.i12h[d];
    }
  }
  {
    // Kreiss-Oliger (symmetric 6th difference) applied to w
    const double wk[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};
    __syncthreads();
    // w is in state layout: stage its interior values
    for (int e = threadIdx.x; e < LX * LY * LZ; e += NT) {
      const int lx = e % LX;
      const int r = e / LX;
      const int ly = r % LY;
      const int lz = r / LY;
      const int qx = tx0 - 3 + lx - 3, qy = ty0 - 3 + ly - 3, qz = tz0 - 3 + lz - 3;
      double v = 0.0;
      if (qx >= 0 && qx < b.nx && qy >= 0 && qy < b.ny && qz >= 0 && qz < b.nz)
        v = w[(int64_t)f * b.fs + (int64_t)(qz + 3) * b.sz + (int64_t)(qy + 3) * b.sy + (qx + 3)];
      t0[e] = v;
    }
    __syncthreads();
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      double sd = 0.0;
#pragma unroll
      for (int o = -3; o <= 3; ++o) sd += wk[o + 3] * t0[c0 - o * st[d]];
      s += sd * b.i64h[d];
    }
    acc += ko_sigma * s;
  }
  if (valid) ubar[(int64_t)f * b.fs + (int64_t)Z * b.sz + (int64_t)Y * b.sy + X] += acc;
}

}  // namespace grf
