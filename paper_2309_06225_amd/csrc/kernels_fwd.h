// Forward kernels of libgrf: LDS-tiled stencil stage, pointwise right-hand side
// fused with the RK4 stage update, periodic ghost fill, status word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen/gen_layout.h"

namespace grf {

constexpr int NF = 27;
constexpr int NG = 3;
constexpr int F_CHI = 0, F_LAPSE = 18, F_SHIFT = 19, F_B = 22;

// Geometry of one box as the kernels see it.
struct BoxDev {
  int nx, ny, nz;
  int ng;          // ghost layers (3; 4 for the sixth-order scheme with eighth-difference dissipation)
  int sy;          // state stride in y (nx + 2 ng)
  int64_t sz;      // state stride in z ((nx + 2 ng)(ny + 2 ng))
  int64_t fs;      // field stride of the state
  int64_t ncell;   // nx*ny*nz
  int64_t as;      // field stride of the compact accumulator: ncell, or the
                   // whole box's cell count when a z-slab of it is processed
  double i12h[3];  // 1/(12 h)
  double i12h2[3]; // 1/(12 h^2)
  double i144[3];  // 1/(144 h_x h_y), 1/(144 h_x h_z), 1/(144 h_y h_z)
  double i64h[3];  // 1/(64 h)
  double i60h[3];    // 1/(60 h)            (sixth-order stencils)
  double i180h2[3];  // 1/(180 h^2)
  double i3600[3];   // 1/(3600 h_x h_y), 1/(3600 h_x h_z), 1/(3600 h_y h_z)
  double i256h[3];   // 1/(256 h)           (eighth-difference dissipation)
};

__device__ __forceinline__ bool advected(int f, int shift_adv) {
  return (f < F_SHIFT || f >= F_B + 3) || shift_adv;
}


// Stencil sums on a line L[0..6] = u at offsets -3..3.  Each sum is taken in
// increasing offset order with every product rounded on its own (no fused
// multiply-add), so that the large cancellation of an O(1) background is
// reproduced exactly; the scale 1/(12 h) etc. is applied afterwards.
#pragma clang fp contract(off)
__device__ __forceinline__ double sten_d1(const double* L) {  // 1, -8, 0, 8, -1
  return ((L[1] - 8.0 * L[2]) + 8.0 * L[4]) - L[5];
}
__device__ __forceinline__ double sten_d2(const double* L) {  // -1, 16, -30, 16, -1
  return ((((-L[1]) + 16.0 * L[2]) - 30.0 * L[3]) + 16.0 * L[4]) - L[5];
}
__device__ __forceinline__ double sten_up_plus(const double* L) {  // offsets -1..3: -3, -10, 18, -6, 1
  return ((((-3.0) * L[2] - 10.0 * L[3]) + 18.0 * L[4]) - 6.0 * L[5]) + L[6];
}
__device__ __forceinline__ double sten_up_minus(const double* L) {  // offsets 1, 0, -1, -2, -3: 3, 10, -18, 6, -1
  return (((3.0 * L[4] + 10.0 * L[3]) - 18.0 * L[2]) + 6.0 * L[1]) - L[0];
}
__device__ __forceinline__ double sten_ko(const double* L) {  // 1, -6, 15, -20, 15, -6, 1
  return (((((L[0] - 6.0 * L[1]) + 15.0 * L[2]) - 20.0 * L[3]) + 15.0 * L[4]) - 6.0 * L[5]) + L[6];
}
// 16-point mixed derivative of the axis pair PAIR (0: x-y, 1: x-z, 2: y-z):
// sum over a (first axis, outer) and b (second axis, inner) of c_a c_b u(a, b),
// c = (1, -8, 0, 8, -1); the weights are powers of two, so every product is
// exact.  Staged values are addressed as t[pb[dz + 3] + cxy + dy * LX + dx].
template <int LX, int PAIR>
__device__ __forceinline__ double sten_mixed(const double* t, const int* pb, int cxy) {
  const double w[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
  double s = 0.0;
#pragma unroll
  for (int a = -2; a <= 2; ++a) {
    if (a == 0) continue;
#pragma unroll
    for (int bb = -2; bb <= 2; ++bb) {
      if (bb == 0) continue;
      const int e = PAIR == 0 ? pb[3] + cxy + bb * LX + a : PAIR == 1 ? pb[bb + 3] + cxy + a : pb[bb + 3] + cxy + a * LX;
      s += (w[a + 2] * w[bb + 2]) * t[e];
    }
  }
  return s;
}
// Sixth-order forms on the same seven points: centred first derivative
// (-1, 9, -45, 0, 45, -9, 1)/(60 h), second derivative
// (2, -27, 270, -490, 270, -27, 2)/(180 h^2), the 36-point mixed derivative
// from the first-derivative weights along both axes / (3600 h_a h_b), and the
// fifth-order advection stencil leaning one cell to the side the shift
// points to: offsets -2..3 with (3, -30, -20, 60, -15, 2)/(60 h) for beta >= 0,
// its mirror image for beta < 0.  All weights and their products are exact.
__device__ __forceinline__ double sten6_d1(const double* L) {
  return ((((-L[0] + 9.0 * L[1]) - 45.0 * L[2]) + 45.0 * L[4]) - 9.0 * L[5]) + L[6];
}
__device__ __forceinline__ double sten6_d2(const double* L) {
  return (((((2.0 * L[0] - 27.0 * L[1]) + 270.0 * L[2]) - 490.0 * L[3]) + 270.0 * L[4]) - 27.0 * L[5]) + 2.0 * L[6];
}
__device__ __forceinline__ double sten6_up_plus(const double* L) {
  return ((((3.0 * L[1] - 30.0 * L[2]) - 20.0 * L[3]) + 60.0 * L[4]) - 15.0 * L[5]) + 2.0 * L[6];
}
__device__ __forceinline__ double sten6_up_minus(const double* L) {
  return ((((-3.0 * L[5] + 30.0 * L[4]) + 20.0 * L[3]) - 60.0 * L[2]) + 15.0 * L[1]) - 2.0 * L[0];
}
// (H: the staged halo, 3 or 4; pb[dz + H] is the plane at z offset dz)
template <int LX, int PAIR, int H = 3>
__device__ __forceinline__ double sten6_mixed(const double* t, const int* pb, int cxy) {
  const double w[7] = {-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0};
  double s = 0.0;
#pragma unroll
  for (int a = -3; a <= 3; ++a) {
    if (a == 0) continue;
#pragma unroll
    for (int bb = -3; bb <= 3; ++bb) {
      if (bb == 0) continue;
      const int e = PAIR == 0 ? pb[H] + cxy + bb * LX + a : PAIR == 1 ? pb[bb + H] + cxy + a : pb[bb + H] + cxy + a * LX;
      s += (w[a + 3] * w[bb + 3]) * t[e];
    }
  }
  return s;
}
// With four ghost layers, on a line L[0..8] = u at offsets -4..4: the
// sixth-order advection stencil leaning one cell to the side the shift points
// to, offsets -2..4 with (2, -24, -35, 80, -30, 8, -1)/(60 h) for beta >= 0 and
// its mirror image for beta < 0, and the eighth difference
// (1, -8, 28, -56, 70, -56, 28, -8, 1), which the dissipation takes with
// weight -sigma/(256 h).
__device__ __forceinline__ double sten6_up7_plus(const double* L) {
  return (((((2.0 * L[2] - 24.0 * L[3]) - 35.0 * L[4]) + 80.0 * L[5]) - 30.0 * L[6]) + 8.0 * L[7]) - L[8];
}
__device__ __forceinline__ double sten6_up7_minus(const double* L) {
  return (((((-2.0 * L[6] + 24.0 * L[5]) + 35.0 * L[4]) - 80.0 * L[3]) + 30.0 * L[2]) - 8.0 * L[1]) + L[0];
}
__device__ __forceinline__ double sten_ko8(const double* L) {
  return (((((((L[0] - 8.0 * L[1]) + 28.0 * L[2]) - 56.0 * L[3]) + 70.0 * L[4]) - 56.0 * L[5]) + 28.0 * L[6]) -
          8.0 * L[7]) + L[8];
}
#pragma clang fp contract(fast)

// ---------------------------------------------------------------------------
// Stencil stage.  One workgroup = one field of one TX*TY*TZ tile.  The tile and
// its 3-deep halo are staged in LDS with coalesced row loads, then every thread
// produces, for its cell, the derivative record of that field:
//   centred d_k (4th order), d_k d_k and the 16-point mixed d_k d_l,
//   the upwinded advection sum beta^k D^up_k u (side by the sign of beta^k),
//   sigma * sum_k (6th difference)/(64 h_k)  (Kreiss-Oliger).
// Output record: D[comp * ncell + cell], cell = (k*ny + j)*nx + i.
// With UP non-null the three upwinded derivatives are also stored (for the VJP):
//   UP[(3 f + k) * ncell + cell].
// Load one field of a tile (interior origin tx0, ty0, tz0) and its 3-deep halo
// into t (coalesced rows); cells beyond the stored box are left untouched.
template <int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void stage_tile(const BoxDev& b, int tx0, int ty0, int tz0, const double* __restrict__ uf,
                                           double* t) {
  constexpr int LX = TX + 6, LY = TY + 6, LZ = TZ + 6;
  for (int e = threadIdx.x; e < LX * LY * LZ; e += NT) {
    const int lx = e % LX;
    const int r = e / LX;
    const int ly = r % LY;
    const int lz = r / LY;
    const int gx = tx0 + lx, gy = ty0 + ly, gz = tz0 + lz;
    if (gx < b.nx + 6 && gy < b.ny + 6 && gz < b.nz + 6) t[e] = uf[(int64_t)gz * b.sz + (int64_t)gy * b.sy + gx];
  }
}

__device__ __forceinline__ void tile_origin(const BoxDev& b, int tile, int TX, int TY, int TZ, int& tx0, int& ty0,
                                            int& tz0) {
  const int ntx = (b.nx + TX - 1) / TX, nty = (b.ny + TY - 1) / TY;
  tx0 = (tile % ntx) * TX;
  tile /= ntx;
  ty0 = (tile % nty) * TY;
  tz0 = (tile / nty) * TZ;
}

// Store of one record component: streamed (non-temporal), the record of a
// whole box goes to memory and is read back by a later kernel.
__device__ __forceinline__ void rec_store(double* p, double v) { __builtin_nontemporal_store(v, p); }

// Derivative record of field f for one cell (interior i, j, k) from staged
// values.  The staged neighbourhood is addressed as t[pb[dz + 3] + cxy + dy*LX + dx]
// (pb: base of the plane at z offset dz, cxy: the cell within a plane), so the
// same arithmetic serves a 3-D tile and a ring of z-planes.  Record layout:
// component q of the cell lives at Dc[q * nc].
// H: the staged halo (3, or 4 for the sixth-order scheme with four ghost
// layers: sixth-order advection and eighth-difference dissipation).
template <int LX, int ORD = 4, int H = 3>
__device__ __forceinline__ void compute_cell(const BoxDev& b, int i, int j, int k, int f, const double* __restrict__ u,
                                             double* __restrict__ Dc, int64_t nc, int64_t cell, double ko_sigma,
                                             int shift_adv, double* __restrict__ UP, const double* t, const int* pb,
                                             int cxy) {
  static_assert(H == 3 || (H == 4 && ORD == 6), "four ghost layers only with the sixth-order scheme");
#define GRF_AT(dx, dy, dz) t[pb[(dz) + H] + cxy + (dy) * LX + (dx)]
  double line[3][2 * H + 1];
#pragma unroll
  for (int o = -H; o <= H; ++o) {
    line[0][o + H] = GRF_AT(o, 0, 0);
    line[1][o + H] = GRF_AT(0, o, 0);
    line[2][o + H] = GRF_AT(0, 0, o);
  }
  // the seven points -3..3 of each line
  const double* l7[3] = {line[0] + (H - 3), line[1] + (H - 3), line[2] + (H - 3)};
  const int s1 = grf_d1_slot[f];
  if (s1 >= 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = ORD == 6 ? sten6_d1(l7[d]) * b.i60h[d] : sten_d1(l7[d]) * b.i12h[d];
      rec_store(&Dc[(int64_t)(GRF_OFF_D1 + 3 * s1 + d) * nc], v);
    }
  }
  const int s2 = grf_d2_slot[f];
  if (s2 >= 0) {
    const int pure[3] = {0, 3, 5};
    if constexpr (ORD == 6) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
        rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + pure[d]) * nc], sten6_d2(l7[d]) * b.i180h2[d]);
      rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + 1) * nc], sten6_mixed<LX, 0, H>(t, pb, cxy) * b.i3600[0]);
      rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + 2) * nc], sten6_mixed<LX, 1, H>(t, pb, cxy) * b.i3600[1]);
      rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + 4) * nc], sten6_mixed<LX, 2, H>(t, pb, cxy) * b.i3600[2]);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d)
        rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + pure[d]) * nc], sten_d2(l7[d]) * b.i12h2[d]);
      rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + 1) * nc], sten_mixed<LX, 0>(t, pb, cxy) * b.i144[0]);
      rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + 2) * nc], sten_mixed<LX, 1>(t, pb, cxy) * b.i144[1]);
      rec_store(&Dc[(int64_t)(GRF_OFF_D2 + 6 * s2 + 4) * nc], sten_mixed<LX, 2>(t, pb, cxy) * b.i144[2]);
    }
  }
#undef GRF_AT
  // upwinded advection: the lopsided stencil on the side the shift points to
  const int64_t sc = (int64_t)(k + H) * b.sz + (int64_t)(j + H) * b.sy + (i + H);
  double beta[3], up[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    beta[d] = u[(int64_t)(F_SHIFT + d) * b.fs + sc];
    if constexpr (H == 4)
      up[d] = (beta[d] >= 0.0 ? sten6_up7_plus(line[d]) : sten6_up7_minus(line[d])) * b.i60h[d];
    else if constexpr (ORD == 6)
      up[d] = (beta[d] >= 0.0 ? sten6_up_plus(l7[d]) : sten6_up_minus(l7[d])) * b.i60h[d];
    else
      up[d] = (beta[d] >= 0.0 ? sten_up_plus(l7[d]) : sten_up_minus(l7[d])) * b.i12h[d];
    if (UP) UP[(int64_t)(3 * f + d) * b.ncell + cell] = up[d];
  }
  // a field whose advection sum enters only its own right-hand side, with
  // coefficient 1, has it added to its Kreiss-Oliger term (one stored value)
  const bool merged = grf_adv_merged[shift_adv != 0][f] != 0;
  double adv = 0.0;
  if (advected(f, shift_adv)) {
    adv = beta[0] * up[0] + beta[1] * up[1] + beta[2] * up[2];
    if (!merged) rec_store(&Dc[(int64_t)(GRF_OFF_ADV + f) * nc], adv);
  }
  double ko = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if constexpr (H == 4)
      ko += (-sten_ko8(line[d])) * b.i256h[d];
    else
      ko += sten_ko(l7[d]) * b.i64h[d];
  }
  rec_store(&Dc[(int64_t)(GRF_OFF_KO + f) * nc], merged ? adv + ko_sigma * ko : ko_sigma * ko);
}

// Derivative record of field f for this thread's cell of a staged 3-D tile
// (D[q * ncell + cell], cell the interior cell index).  Threads outside the box
// do nothing.
template <int TX, int TY, int TZ>
__device__ __forceinline__ void compute_tile(const BoxDev& b, int tx0, int ty0, int tz0, int f,
                                             const double* __restrict__ u, double* __restrict__ D, double ko_sigma,
                                             int shift_adv, double* __restrict__ UP, const double* t) {
  constexpr int LX = TX + 6, LY = TY + 6;
  const int ix = threadIdx.x % TX;
  const int iy = (threadIdx.x / TX) % TY;
  const int iz = threadIdx.x / (TX * TY);
  const int i = tx0 + ix, j = ty0 + iy, k = tz0 + iz;
  if (i >= b.nx || j >= b.ny || k >= b.nz) return;
  const int64_t cell = ((int64_t)k * b.ny + j) * b.nx + i;
  int pb[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) pb[o] = (iz + o) * LX * LY;
  const int cxy = (iy + 3) * LX + (ix + 3);
  compute_cell<LX>(b, i, j, k, f, u, D + cell, b.ncell, cell, ko_sigma, shift_adv, UP, t, pb, cxy);
}

template <int TX, int TY, int TZ>
__device__ __forceinline__ void deriv_tile(const BoxDev& b, int tile, int f, const double* __restrict__ u,
                                           double* __restrict__ D, double ko_sigma, int shift_adv,
                                           double* __restrict__ UP, double* t) {
  int tx0, ty0, tz0;
  tile_origin(b, tile, TX, TY, TZ, tx0, ty0, tz0);
  __syncthreads();  // the previous work item of this workgroup is done with t
  stage_tile<TX, TY, TZ, TX * TY * TZ>(b, tx0, ty0, tz0, u + (int64_t)f * b.fs, t);
  __syncthreads();
  compute_tile<TX, TY, TZ>(b, tx0, ty0, tz0, f, u, D, ko_sigma, shift_adv, UP, t);
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_deriv(BoxDev b, const double* __restrict__ u,
                                                      double* __restrict__ D, double ko_sigma, int shift_adv,
                                                      double* __restrict__ UP) {
  __shared__ double t[(TZ + 6) * (TY + 6) * (TX + 6)];
  deriv_tile<TX, TY, TZ>(b, blockIdx.x, blockIdx.y, u, D, ko_sigma, shift_adv, UP, t);
}

// Stencil stage, z-marching form.  One workgroup = one field of a TX*TY column
// of cells over a chunk of ZC z-planes.  The workgroup walks up the column with a
// ring of 8 LDS planes (each TX+6 by TY+6): every step loads one new plane and
// computes one plane of cells from the 7 planes around it, so each plane of the
// field is read from memory once per column instead of once per overlapping
// tile.  With 8 slots for a 7-plane stencil, one barrier per step suffices: the
// slot a step writes is never one the previous step reads.  The global loads of
// the next plane are in flight while the current plane is computed.
// Work-item order with XCDMAP: consecutive items are the 27 fields of one column
// chunk, and the hardware's round-robin dealing of workgroups over the 8 XCDs
// is undone so that consecutive items share an XCD, and with it the L2 that
// holds the column's shift values and the halo of the previous column.
__device__ __forceinline__ int xcd_item(int w, int nblocks) {
  const int per = nblocks >> 3, rem = nblocks & 7;
  const int x = w & 7, s = w >> 3;
  return x * per + (x < rem ? x : rem) + s;
}

// Number of (column, z-chunk) items of a box for the z-marching form.
template <int TX, int TY, int ZC>
__host__ __device__ inline int zm_items(const BoxDev& b) {
  return ((b.nx + TX - 1) / TX) * ((b.ny + TY - 1) / TY) * ((b.nz + ZC - 1) / ZC);
}

// One field of one (column, z-chunk) item: item = column x + ntx (column y +
// nty chunk).  t: zm_ring(H) * (TX+2H)(TY+2H) doubles of LDS, H the halo.
// A ring of 2H + 2 planes for a (2H + 1)-plane stencil needs one barrier per
// step (the slot a step writes is never one the previous step reads).
__host__ __device__ constexpr int zm_ring(int h) { return 2 * h + 2; }

template <int TX, int TY, int ZC, int ORD = 4, int H = 3>
__device__ __forceinline__ void zm_column(const BoxDev& b, int item, int f, const double* __restrict__ u,
                                          double* __restrict__ D, double ko_sigma, int shift_adv,
                                          double* __restrict__ UP, double* t) {
  constexpr int LX = TX + 2 * H, LY = TY + 2 * H, PL = LX * LY, NT = TX * TY, R = zm_ring(H);
  const int ntx = (b.nx + TX - 1) / TX, nty = (b.ny + TY - 1) / TY;
  const int tx0 = (item % ntx) * TX;
  item /= ntx;
  const int ty0 = (item % nty) * TY;
  const int z0 = (item / nty) * ZC;
  const int z1 = min(z0 + ZC, b.nz);
  const double* __restrict__ uf = u + (int64_t)f * b.fs;
  const int ix = threadIdx.x % TX, iy = threadIdx.x / TX;
  const int i = tx0 + ix, j = ty0 + iy;
  const bool inside = i < b.nx && j < b.ny;
  const int cxy = (iy + H) * LX + (ix + H);
  // a plane of the column (ghost-inclusive z = gz) is fetched into registers,
  // PER values per thread, and later written to its ring slot gz mod R; the
  // fetch of the next plane is issued before the current plane is computed
  constexpr int PER = (PL + NT - 1) / NT;
  double pre[PER];
  auto fetch_plane = [&](int gz) {
    const double* up = uf + (int64_t)gz * b.sz;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NT;
      const int lx = e % LX, ly = e / LX;
      const int gx = tx0 + lx, gy = ty0 + ly;
      pre[q] = (e < PL && gx < b.nx + 2 * H && gy < b.ny + 2 * H) ? up[(int64_t)gy * b.sy + gx] : 0.0;
    }
  };
  auto store_plane = [&](int gz) {
    double* tp = t + ((unsigned)gz % R) * PL;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < PL) tp[e] = pre[q];
    }
  };
  __syncthreads();  // an earlier item of this workgroup is done with t
  for (int gz = z0; gz < z0 + 2 * H; ++gz) {
    fetch_plane(gz);
    store_plane(gz);
  }
  fetch_plane(z0 + 2 * H);
  for (int k = z0; k < z1; ++k) {
    store_plane(k + 2 * H);
    __syncthreads();
    if (k + 1 < z1) fetch_plane(k + 2 * H + 1);
    if (inside) {
      int pb[2 * H + 1];
#pragma unroll
      for (int o = 0; o < 2 * H + 1; ++o) pb[o] = ((unsigned)(k + o) % R) * PL;
      const int64_t cell = ((int64_t)k * b.ny + j) * b.nx + i;
      compute_cell<LX, ORD, H>(b, i, j, k, f, u, D + cell, b.ncell, cell, ko_sigma, shift_adv, UP, t, pb,
                                     cxy);
    }
  }
}

template <int TX, int TY, int ZC, bool XCDMAP, int ORD = 4, int H = 3>
__global__ __launch_bounds__(TX* TY) void k_deriv_zm(BoxDev b, const double* __restrict__ u,
                                                      double* __restrict__ D, double ko_sigma, int shift_adv,
                                                      double* __restrict__ UP) {
  __shared__ double t[zm_ring(H) * (TX + 2 * H) * (TY + 2 * H)];
  int item = blockIdx.x, f;
  if (XCDMAP) {
    item = xcd_item(item, (int)gridDim.x);
    f = item % NF;
    item /= NF;
  } else {  // field slowest, as in the tiled form
    const int per_field = (int)gridDim.x / NF;
    f = item / per_field;
    item %= per_field;
  }
  zm_column<TX, TY, ZC, ORD, H>(b, item, f, u, D, ko_sigma, shift_adv, UP, t);
}

// ---------------------------------------------------------------------------
// Pointwise right-hand side (generated algebra) fused with the RK4 stage.
// MODE 0: rhs[f] = k;  MODE 1: first stage;  MODE 2: middle stage;  MODE 4: last stage.
struct StageCoef {
  double cnext;  // c_s dt for stages 1-3, dt/6 for stage 4
};

// RK4 stage update of one field in the textbook order: acc holds
// k1 + 2 k2 + 2 k3 (summed in that order), stage states are u0 + (c dt) k, the
// new state u0 + (dt/6)(acc + k4).  Products are rounded on their own (no fused
// multiply-add) so that states carrying a tiny perturbation on an O(1)
// background round exactly as the textbook formula does.  k includes the
// Kreiss-Oliger term stored by the stencil stage.
#pragma clang fp contract(off)
template <int MODE>
__device__ __forceinline__ void stage_one(int f, double rhs_f, double ko_f, const BoxDev& b, int64_t c, int64_t s,
                                          const double* __restrict__ u0, double* __restrict__ out,
                                          double* __restrict__ acc, StageCoef sc, unsigned& flags) {
  const double kf = rhs_f + ko_f;
  if (!isfinite(kf)) flags |= 1u;
  const int64_t q = (int64_t)f * b.fs + s;
  const int64_t qa = (int64_t)f * b.as + c;
  if constexpr (MODE == 0) {
    out[q] = kf;
  } else if constexpr (MODE == 1) {
    acc[qa] = kf;
    out[q] = u0[q] + sc.cnext * kf;
  } else if constexpr (MODE == 2) {
    acc[qa] = acc[qa] + 2.0 * kf;
    out[q] = u0[q] + sc.cnext * kf;
  } else {
    out[q] = u0[q] + sc.cnext * (acc[qa] + kf);
  }
}
#pragma clang fp contract(fast)

// One interior cell c of box b: right-hand side and stage update (MODE 0: rhs
// only; 1: first stage; 2: middle stage; 4: last stage).
template <int MODE, int SHIFTADV>
__device__ __forceinline__ void point_cell(const BoxDev& b, int64_t c, const grf_point_params& P,
                                           const double* __restrict__ us, const double* __restrict__ D,
                                           int64_t dstride, int64_t dcell, const double* __restrict__ u0,
                                           double* __restrict__ out, double* __restrict__ acc, StageCoef sc,
                                           unsigned* __restrict__ status) {
  const int i = (int)(c % b.nx);
  const int64_t r = c / b.nx;
  const int j = (int)(r % b.ny);
  const int k = (int)(r / b.ny);
  const int64_t s = (int64_t)(k + 3) * b.sz + (int64_t)(j + 3) * b.sy + (i + 3);
  const int64_t nc = b.ncell;
  int bad = 0;
  unsigned flags = 0u;
#define GRF_U(f) us[(int64_t)(f) * b.fs + s]
#define GRF_D(cc) D[(int64_t)(cc) * dstride + dcell]
#define GRF_P(n) P.n
#define GRF_RHS(f, v) \
  stage_one<MODE>(f, (v), D[(int64_t)(GRF_OFF_KO + (f)) * dstride + dcell], b, c, s, u0, out, acc, sc, flags)
#define GRF_PIVCHK(v) bad |= !(fabs(v) <= 1e12)
#define GRF_SHIFT_ADVEC (SHIFTADV != 0)
#include "gen/gen_rhs.inc"
#undef GRF_SHIFT_ADVEC
#undef GRF_RHS
#undef GRF_PIVCHK
#undef GRF_U
#undef GRF_D
#undef GRF_P
  if (bad) flags |= 2u;
  if (!(us[(int64_t)F_CHI * b.fs + s] > 0.0) || !(us[(int64_t)F_LAPSE * b.fs + s] > 0.0)) flags |= 4u;
  if (flags) atomicOr(status, flags);
}

constexpr int kPointThreads = 128;

template <int MODE, int SHIFTADV>
__global__ __launch_bounds__(kPointThreads) void k_point(BoxDev b, grf_point_params P, const double* __restrict__ us,
                                                         const double* __restrict__ D,
                                                         const double* __restrict__ u0, double* __restrict__ out,
                                                         double* __restrict__ acc, StageCoef sc,
                                                         unsigned* __restrict__ status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.ncell) return;
  point_cell<MODE, SHIFTADV>(b, c, P, us, D, b.ncell, c, u0, out, acc, sc, status);
}

}  // namespace grf
