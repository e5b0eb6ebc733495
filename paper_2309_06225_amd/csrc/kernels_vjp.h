// Reverse-mode kernels of libgrf: vector-Jacobian product of the right-hand side.
//
// Pass 1 (k_deriv with UP): derivative record D and upwinded derivatives UP at u.
// Pass 2 (k_vjp_point): per interior cell, the generated reverse of the pointwise
//   algebra.  Given w (cotangent of the right-hand side) it adds the cotangent of
//   the cell's own field values to u_bar, stores the cotangents of every stencil
//   input (first/second derivatives, advection sums) in Dbar, adds the shift's
//   share of the advection sums (sum_f adv_bar_f * D^up_k u_f) to u_bar, and
//   stores the cell's coupling cotangents in TH.
// Pass 3 (k_vjp_gather): for every cell of the box, ghosts included, gathers
//   the transposed stencils: sum over interior source cells c of stencil weight
//   times the cotangent stored at c (and the Kreiss-Oliger stencil applied to w).
// Pass 4 (k_reduce_*): fixed-order tree sum of TH into theta_bar.
#pragma once
#include "kernels_fwd.h"

namespace grf {

constexpr int NTH = 2;
// components of the cotangent record Dbar (same numbering as D, without Kreiss-Oliger)
constexpr int NCOMP_BAR = GRF_OFF_KO;

// Two waves per SIMD (256 registers each): the kernel spills ~12 KB per lane
// either way, and the second wave hides part of that traffic's latency
// (3.86 -> 3.04 ms at 64^3; three or four waves per SIMD measured slower).
// DEC: the decoupling limit (the scalar does not source the metric).
template <int SHIFTADV, int DEC = 0>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_vjp_point(BoxDev b, grf_point_params P, const double* __restrict__ us,
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
  if constexpr (DEC != 0) {
#include "gen/gen_vjp_dec.inc"
  } else {
#include "gen/gen_vjp.inc"
  }
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
      // the cotangent of a field's advection sum: w_f where the sum is carried
      // in the Kreiss-Oliger slot, else the generated code's value
      const double abar = grf_adv_merged[SHIFTADV != 0][f] ? w[(int64_t)f * b.fs + s]
                                                           : Dbar[(int64_t)(GRF_OFF_ADV + f) * nc + c];
      sb += abar * UP[(int64_t)(3 * f + d) * nc + c];
    }
    ub[F_SHIFT + d] += sb;
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) ubar[(int64_t)f * b.fs + s] += ub[f];
}

// Pass 3, transposed stencils in gather form: one thread per (cell of the full
// box incl. ghosts, field), every source value read from memory through the
// caches (a wave's cells are consecutive in x, so each stencil point is one
// contiguous row read); sources outside the interior contribute nothing.
// u_bar[f] += sum over the field's stencils of their transposes applied to the
// cotangent record (the upwind split by the sign of the shift at the source
// cell) and the Kreiss-Oliger transpose applied to w.  Every load is issued
// unconditionally (see src_at), so a thread's loads of one stencil group are
// in flight together; with a bounds branch around each load they were issued
// and waited for one at a time (1.06 ms at 64^3 against 0.55).  (An LDS-tiled
// form of the same sums measured 1.30 ms.)  ORD 6: the transposes
// of the sixth-order stencils of the three-ghost box (centred derivatives on
// seven points, the fifth-order biased advection stencils), the same
// Kreiss-Oliger operator; with H = 4 (four ghost layers) the sixth-order
// biased stencils on seven points and the eighth difference.
// (X, Y, Z: state coordinates on a box with H ghost layers)
// The load is unconditional, from the source clamped into the interior (always
// in bounds), and the value is dropped afterwards when the source lies
// outside: no branch per load, so a thread issues all its loads before it
// waits for any.
__device__ __forceinline__ int clamp_to(int v, int n) { return min(max(v, 0), n - 1); }

// (bitwise ands: no short-circuit branches for the compiler to sink the loads into)
__device__ __forceinline__ bool inside(const BoxDev& b, int ix, int iy, int iz) {
  return (ix >= 0) & (ix < b.nx) & (iy >= 0) & (iy < b.ny) & (iz >= 0) & (iz < b.nz);
}

template <int H = 3>
__device__ __forceinline__ double src_at(const BoxDev& b, const double* __restrict__ comp, int X, int Y, int Z) {
  const int ix = X - H, iy = Y - H, iz = Z - H;
  const double v =
      comp[((int64_t)clamp_to(iz, b.nz) * b.ny + clamp_to(iy, b.ny)) * b.nx + clamp_to(ix, b.nx)];
  return inside(b, ix, iy, iz) ? v : 0.0;
}

constexpr int kGatherThreads = 512;  // 0.50 ms per 64^3 gather against 0.56 with 128 or 256 and 0.55 with 1024

template <int NT, int ORD = 4, int H = 3>
__global__ __launch_bounds__(NT) void k_vjp_gather(BoxDev b, const double* __restrict__ u,
                                                               const double* __restrict__ w,
                                                               const double* __restrict__ Dbar, double ko_sigma,
                                                               int shift_adv, double* __restrict__ ubar) {
  static_assert(H == 3 || (H == 4 && ORD == 6), "four ghost layers only with the sixth-order scheme");
  const int f = blockIdx.y;
  const int NX = b.nx + 2 * H, NY = b.ny + 2 * H, NZ = b.nz + 2 * H;
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)NX * NY * NZ) return;
  const int X = (int)(e % NX);
  const int64_t r = e / NX;
  const int Y = (int)(r % NY), Z = (int)(r / NY);
  const int64_t nc = b.ncell;
  auto at = [&](const double* comp, int d, int o) {  // comp at the target moved by -o along d
    return src_at<H>(b, comp, X - (d == 0 ? o : 0), Y - (d == 1 ? o : 0), Z - (d == 2 ? o : 0));
  };
  double acc = 0.0;
  const int s1 = grf_d1_slot[f];
  const int s2 = grf_d2_slot[f];
  if constexpr (ORD == 6) {
    const double w1[7] = {-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0};
    const double w2[7] = {2.0, -27.0, 270.0, -490.0, 270.0, -27.0, 2.0};
    if (s1 >= 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double* comp = Dbar + (int64_t)(GRF_OFF_D1 + 3 * s1 + d) * nc;
        double s = 0.0;
#pragma unroll
        for (int o = -3; o <= 3; ++o)
          if (o != 0) s += w1[o + 3] * at(comp, d, o);
        acc += s * b.i60h[d];
      }
    }
    if (s2 >= 0) {
      const int pure[3] = {0, 3, 5};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double* comp = Dbar + (int64_t)(GRF_OFF_D2 + 6 * s2 + pure[d]) * nc;
        double s = 0.0;
#pragma unroll
        for (int o = -3; o <= 3; ++o) s += w2[o + 3] * at(comp, d, o);
        acc += s * b.i180h2[d];
      }
      const int pd[3] = {0, 0, 1}, pe[3] = {1, 2, 2}, pq[3] = {1, 2, 4};
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double* comp = Dbar + (int64_t)(GRF_OFF_D2 + 6 * s2 + pq[m]) * nc;
        double s = 0.0;
#pragma unroll
        for (int a = -3; a <= 3; ++a)
#pragma unroll
          for (int bb = -3; bb <= 3; ++bb)
            if (a != 0 && bb != 0) {
              int dx[3] = {0, 0, 0};
              dx[pd[m]] += a;
              dx[pe[m]] += bb;
              s += (w1[a + 3] * w1[bb + 3]) * src_at<H>(b, comp, X - dx[0], Y - dx[1], Z - dx[2]);
            }
        acc += s * b.i3600[m];
      }
    }
  } else {
  if (s1 >= 0) {
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* comp = Dbar + (int64_t)(GRF_OFF_D1 + 3 * s1 + d) * nc;
      double s = 0.0;
#pragma unroll
      for (int o = -2; o <= 2; ++o)
        if (o != 0) s += w1[o + 2] * at(comp, d, o);
      acc += s * b.i12h[d];
    }
  }
  if (s2 >= 0) {
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
    const double w2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    const int pure[3] = {0, 3, 5};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* comp = Dbar + (int64_t)(GRF_OFF_D2 + 6 * s2 + pure[d]) * nc;
      double s = 0.0;
#pragma unroll
      for (int o = -2; o <= 2; ++o) s += w2[o + 2] * at(comp, d, o);
      acc += s * b.i12h2[d];
    }
    const int pd[3] = {0, 0, 1}, pe[3] = {1, 2, 2}, pq[3] = {1, 2, 4};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double* comp = Dbar + (int64_t)(GRF_OFF_D2 + 6 * s2 + pq[m]) * nc;
      double s = 0.0;
#pragma unroll
      for (int a = -2; a <= 2; ++a)
#pragma unroll
        for (int bb = -2; bb <= 2; ++bb)
          if (a != 0 && bb != 0) {
            int dx[3] = {0, 0, 0};
            dx[pd[m]] += a;
            dx[pe[m]] += bb;
            s += (w1[a + 2] * w1[bb + 2]) * src_at(b, comp, X - dx[0], Y - dx[1], Z - dx[2]);
          }
      acc += s * b.i144[m];
    }
  }
  }  // ORD 4
  if (advected(f, shift_adv)) {
    // forward weights of the biased stencils at offsets -H..H from the source
    // cell, for a nonnegative (wp) and a negative (wm) shift there
    double wp[2 * H + 1], wm[2 * H + 1];
    if constexpr (H == 4) {
      const double p7[9] = {0.0, 0.0, 2.0, -24.0, -35.0, 80.0, -30.0, 8.0, -1.0};
      const double m7[9] = {1.0, -8.0, 30.0, -80.0, 35.0, 24.0, -2.0, 0.0, 0.0};
      for (int q = 0; q < 9; ++q) wp[q] = p7[q], wm[q] = m7[q];
    } else if constexpr (ORD == 6) {
      const double p6[7] = {0.0, 3.0, -30.0, -20.0, 60.0, -15.0, 2.0};
      const double m6[7] = {-2.0, 15.0, -60.0, 20.0, 30.0, -3.0, 0.0};
      for (int q = 0; q < 7; ++q) wp[q] = p6[q], wm[q] = m6[q];
    } else {
      const double p4[7] = {0.0, 0.0, -3.0, -10.0, 18.0, -6.0, 1.0};
      const double m4[7] = {-1.0, 6.0, -18.0, 10.0, 3.0, 0.0, 0.0};
      for (int q = 0; q < 7; ++q) wp[q] = p4[q], wm[q] = m4[q];
    }
    const double* comp = Dbar + (int64_t)(GRF_OFF_ADV + f) * nc;
    // the advection sum's cotangent: w_f where the sum rides in the
    // Kreiss-Oliger slot, else the cotangent record
    const bool merged = grf_adv_merged[shift_adv != 0][f] != 0;
    const double* wf_adv = w + (int64_t)f * b.fs;
    for (int d = 0; d < 3; ++d) {
      const double* beta = u + (int64_t)(F_SHIFT + d) * b.fs;
      double s = 0.0;
#pragma unroll
      for (int o = -H; o <= H; ++o) {
        const int ix = X - (d == 0 ? o : 0) - H, iy = Y - (d == 1 ? o : 0) - H, iz = Z - (d == 2 ? o : 0) - H;
        const bool in = inside(b, ix, iy, iz);
        const int cx = clamp_to(ix, b.nx), cy = clamp_to(iy, b.ny), cz = clamp_to(iz, b.nz);
        const int64_t st = (int64_t)(cz + H) * b.sz + (int64_t)(cy + H) * b.sy + (cx + H);
        const double a = merged ? wf_adv[st] : comp[((int64_t)cz * b.ny + cy) * b.nx + cx];
        const double bd = beta[st];
        const double ab = a * bd;
        const double vp = (in & (bd >= 0.0)) ? ab : 0.0;
        const double vm = (in & !(bd >= 0.0)) ? ab : 0.0;
        s += wp[o + H] * vp + wm[o + H] * vm;
      }
      acc += s * (ORD == 6 ? b.i60h[d] : b.i12h[d]);
    }
  }
  {
    // Kreiss-Oliger (symmetric): the sixth difference over 64 h, or with four
    // ghost layers minus the eighth difference over 256 h
    double wk[2 * H + 1];
    if constexpr (H == 4) {
      const double k8[9] = {1.0, -8.0, 28.0, -56.0, 70.0, -56.0, 28.0, -8.0, 1.0};
      for (int q = 0; q < 9; ++q) wk[q] = k8[q];
    } else {
      const double k6[7] = {1.0, -6.0, 15.0, -20.0, 15.0, -6.0, 1.0};
      for (int q = 0; q < 7; ++q) wk[q] = k6[q];
    }
    const double* wf = w + (int64_t)f * b.fs;
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      double sd = 0.0;
#pragma unroll
      for (int o = -H; o <= H; ++o) {
        const int ix = X - (d == 0 ? o : 0) - H, iy = Y - (d == 1 ? o : 0) - H, iz = Z - (d == 2 ? o : 0) - H;
        const double v = wf[(int64_t)(clamp_to(iz, b.nz) + H) * b.sz + (int64_t)(clamp_to(iy, b.ny) + H) * b.sy +
                            (clamp_to(ix, b.nx) + H)];
        sd += wk[o + H] * (inside(b, ix, iy, iz) ? v : 0.0);
      }
      s += sd * (H == 4 ? -b.i256h[d] : b.i64h[d]);
    }
    acc += ko_sigma * s;
  }
  ubar[(int64_t)f * b.fs + (int64_t)Z * b.sz + (int64_t)Y * b.sy + X] += acc;
}

}  // namespace grf
