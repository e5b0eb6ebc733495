// Batched kernels: one launch per RK4 stage phase covers every box of a batch.
// Work lists are static (box, tile) and (box, cell block) entries; workgroup w
// takes entries w, w + G, w + 2G, ... (G the grid: one workgroup per entry as
// launched, a persistent grid works the same way), so no atomics are involved
// and every cell is computed by exactly the same device code as in the per-box
// launches (results are bitwise identical).
#pragma once
#include "kernels_fwd.h"
#include "kernels_staged.h"

namespace grf {

struct BatchBoxDev {
  BoxDev bd;
  double* u;    // the state (caller's buffer; each step writes its new state here)
  double* ub;   // stage scratch
  double* ua;   // stage scratch
  double* acc;  // compact accumulator
  double* D;    // derivative records
  double dt;
};

struct TileEntry {
  int box;
  int tile;
};
struct CellEntry {  // 64 cells c0 .. c0 + 63 of a box (fewer at its end)
  int box;
  int pad;
  int64_t c0;
};

// Buffer roles of RK4 stage s (1..4): base state, stage input, stage output.
// Every step maps u to u: stage 1 u -> ua, 2 ua -> ub, 3 ub -> ua, 4 ua -> u.
// The last stage writes the new state over its base; that is safe because a
// cell's new value depends on the base only at that cell, and each lane reads
// a cell's base values before it writes them (the stencils of stage 4 read ua).
__device__ __forceinline__ void stage_roles(const BatchBoxDev& B, int stage, const double*& base,
                                            const double*& in, double*& out) {
  base = B.u;
  switch (stage) {
    case 1: in = B.u; out = B.ua; break;
    case 2: in = B.ua; out = B.ub; break;
    case 3: in = B.ub; out = B.ua; break;
    default: in = B.ua; out = B.u; break;
  }
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(TX* TY* TZ) void k_deriv_batch(const BatchBoxDev* __restrict__ boxes,
                                                            const TileEntry* __restrict__ entries, int nentries,
                                                            int stage, double ko_sigma, int shift_adv) {
  __shared__ double t[(TZ + 6) * (TY + 6) * (TX + 6)];
  const int64_t total = (int64_t)nentries * NF;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int e = (int)(g / NF), f = (int)(g % NF);
    const TileEntry en = entries[e];
    const BatchBoxDev B = boxes[en.box];
    const double *base, *in;
    double* out;
    stage_roles(B, stage, base, in, out);
    deriv_tile<TX, TY, TZ>(B.bd, en.tile, f, in, B.D, ko_sigma, shift_adv, nullptr, t);
  }
}

// z-marching stencil stage over (box, column chunk) entries, the 27 fields of
// an entry consecutive.
template <int TX, int TY, int ZC>
__global__ __launch_bounds__(TX* TY) void k_deriv_batch_zm(const BatchBoxDev* __restrict__ boxes,
                                                           const TileEntry* __restrict__ entries, int nentries,
                                                           int stage, double ko_sigma, int shift_adv) {
  __shared__ double t[8 * (TX + 6) * (TY + 6)];
  const int64_t total = (int64_t)nentries * NF;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int e = (int)(g / NF), f = (int)(g % NF);
    const TileEntry en = entries[e];
    const BatchBoxDev B = boxes[en.box];
    const double *base, *in;
    double* out;
    stage_roles(B, stage, base, in, out);
    zm_column<TX, TY, ZC>(B.bd, en.tile, f, in, B.D, ko_sigma, shift_adv, nullptr, t);
  }
}

// Pointwise + RK4 stage over (box, 64-cell block) entries: one wave per
// workgroup and one entry per workgroup (grid = number of entries), with the
// staged inputs of k_point_staged.  A persistent loop over entries here cost
// the kernel ~180 B/lane more spilling (596 against 420) and 13 % of its speed.
template <int MODE, int SHIFTADV>
__global__ __launch_bounds__(kStagedThreads) void k_point_batch(const BatchBoxDev* __restrict__ boxes,
                                                                const CellEntry* __restrict__ entries, int nentries,
                                                                int stage, grf_point_params P,
                                                                unsigned* __restrict__ status) {
  __shared__ double lbuf0_[GRF_STAGE_SLOTS * 64];
  __shared__ double lbuf1_[GRF_STAGE_SLOTS * 64];
  const int g = blockIdx.x;
  if (g >= nentries) return;
  const CellEntry en = entries[g];
  const BatchBoxDev B = boxes[en.box];
  const double *base, *in;
  double* out;
  stage_roles(B, stage, base, in, out);
  StageCoef sc;
  sc.cnext = stage == 4 ? B.dt / 6.0 : (stage == 3 ? 1.0 * B.dt : 0.5 * B.dt);
  staged_wave<MODE, SHIFTADV>(B.bd, en.c0, P, in, B.D, base, out, B.acc, sc, status, (grf_lds_double*)lbuf0_,
                              (grf_lds_double*)lbuf1_);
}

}  // namespace grf
