// Pointwise right-hand side + RK4 stage with asynchronously staged inputs.
//
// The pointwise kernel needs about 250 values per cell from memory (derivative
// record components, the state, u0 and the accumulator) and holds so many
// intermediates that only one wave fits per SIMD, so each load that the
// straight-line code waits for stalls the SIMD.  Here one workgroup is one
// wave of 64 consecutive cells; the generated code is cut into phases of at
// most GRF_STAGE_SLOTS staged items, and while phase j computes from LDS buffer
// j % 2, the items of phase j + 1 are copied from memory into the other buffer
// by LDS-direct loads, which occupy no registers.  A phase boundary waits for
// every outstanding memory operation and LDS read of the wave (so the copies of
// the new phase have landed and nothing still reads the buffer about to be
// refilled) and is fenced against instruction motion.
//
// An item is one double per cell of the wave: two dword copies, the first
// bringing cells 0-31 (lane 2m, 2m+1: low and high word of cell m), the second
// cells 32-63.  Cells past the end of the box read the last cell instead (in
// bounds; they compute and store the last cell's results again).  The
// arithmetic is that of k_point.
#pragma once
#include "kernels_fwd.h"

namespace grf {

typedef __attribute__((address_space(3))) void grf_lds_void;
typedef __attribute__((address_space(3))) double grf_lds_double;
typedef __attribute__((address_space(1))) void grf_global_void;

constexpr int kStagedThreads = 64;
// s_waitcnt with vmcnt(0), expcnt(7), lgkmcnt(0)
constexpr int kWaitAllVmLgkm = 0x0070;

__device__ __forceinline__ int64_t state_offset(const BoxDev& b, int64_t c) {
  const int i = (int)(c % b.nx);
  const int64_t r = c / b.nx;
  const int j = (int)(r % b.ny);
  const int k = (int)(r / b.ny);
  return (int64_t)(k + 3) * b.sz + (int64_t)(j + 3) * b.sy + (i + 3);
}

// Copy one item (64 doubles) into an LDS slot: p0 / p1 point at the double of
// this lane's cell pair for the first / second half of the wave; wb is this
// lane's word offset in bytes (0 or 4).
// AUX: cache policy bits of the load (2: non-temporal, for data read once).
template <int AUX = 0>
__device__ __forceinline__ void stage_item(const double* p0, const double* p1, int wb, grf_lds_double* slot) {
  __builtin_amdgcn_global_load_lds((grf_global_void*)((const char*)p0 + wb), (grf_lds_void*)slot, 4, 0, AUX);
  __builtin_amdgcn_global_load_lds((grf_global_void*)((const char*)p1 + wb), (grf_lds_void*)(slot + 32), 4, 0, AUX);
}

// RK4 stage update of one field from staged values (the order and rounding of
// stage_one), stored non-temporally.
#pragma clang fp contract(off)
template <int MODE>
__device__ __forceinline__ void stage_one_st(int f, double rhs_f, double ko_f, double u0_f, double acc_f,
                                             const BoxDev& b, int64_t c, int64_t s, double* __restrict__ out,
                                             double* __restrict__ acc, StageCoef sc, unsigned& flags) {
  const double kf = rhs_f + ko_f;
  if (!isfinite(kf)) flags |= 1u;
  const int64_t q = (int64_t)f * b.fs + s;
  const int64_t qa = (int64_t)f * b.as + c;
#define GRF_ST(p, v) __builtin_nontemporal_store((v), &(p))
  if constexpr (MODE == 0) {
    GRF_ST(out[q], kf);
  } else if constexpr (MODE == 1) {
    GRF_ST(acc[qa], kf);
    GRF_ST(out[q], u0_f + sc.cnext * kf);
  } else if constexpr (MODE == 2) {
    GRF_ST(acc[qa], acc_f + 2.0 * kf);
    GRF_ST(out[q], u0_f + sc.cnext * kf);
  } else {
    GRF_ST(out[q], u0_f + sc.cnext * (acc_f + kf));
  }
#undef GRF_ST
}
#pragma clang fp contract(fast)

// The 64 cells c0 .. c0 + 63 of box b (one wave; lbuf0 / lbuf1: this wave's
// two LDS buffers of GRF_STAGE_SLOTS items).
template <int MODE, int SHIFTADV, int VAR = 0>
__device__ __forceinline__ void staged_wave(const BoxDev& b, int64_t c0, const grf_point_params& P,
                                            const double* __restrict__ us, const double* __restrict__ D,
                                            const double* __restrict__ u0, double* __restrict__ out,
                                            double* __restrict__ acc, StageCoef sc, unsigned* __restrict__ status,
                                            grf_lds_double* const lbuf0, grf_lds_double* const lbuf1) {
  const int lane = threadIdx.x;
  const int64_t last = b.ncell - 1;
  // lanes past the end of the box redo the last cell: same inputs, same
  // results, so their stores write the bits that the last cell's lane writes
  const int64_t c = min(c0 + lane, last);
  const int64_t s = state_offset(b, c);
  // the cells whose words this lane copies, in the first and second half
  const int64_t vc0 = min(c0 + (lane >> 1), last), vc1 = min(c0 + 32 + (lane >> 1), last);
  const int64_t vs0 = state_offset(b, vc0), vs1 = state_offset(b, vc1);
  const int wb = (lane & 1) * 4;
  const int64_t nc = b.ncell;
  int bad = 0;
  unsigned flags = 0u;
#define GRF_BUF(bb) ((bb) ? lbuf1 : lbuf0)
#define GRF_LDS(bb, slot) GRF_BUF(bb)[(slot) * 64 + lane]
// record components are read once: non-temporal
#define GRF_STAGE_D(bb, slot, cc) \
  stage_item<2>(D + (int64_t)(cc) * nc + vc0, D + (int64_t)(cc) * nc + vc1, wb, &GRF_BUF(bb)[(slot) * 64])
#define GRF_STAGE_KO(bb, slot, f) GRF_STAGE_D(bb, slot, GRF_OFF_KO + (f))
// every input and output of the kernel is read or written once: all of it
// streams past the caches (non-temporal), leaving them to the register spills
#define GRF_STAGE_U(bb, slot, f) \
  stage_item<2>(us + (int64_t)(f) * b.fs + vs0, us + (int64_t)(f) * b.fs + vs1, wb, &GRF_BUF(bb)[(slot) * 64])
#define GRF_STAGE_U0(bb, slot, f)                                                                              \
  do {                                                                                                         \
    if constexpr (MODE != 0)                                                                                   \
      stage_item<2>(u0 + (int64_t)(f) * b.fs + vs0, u0 + (int64_t)(f) * b.fs + vs1, wb, &GRF_BUF(bb)[(slot) * 64]); \
  } while (0)
#define GRF_STAGE_ACC(bb, slot, f)                                                                         \
  do {                                                                                                     \
    if constexpr (MODE == 2 || MODE == 4)                                                                  \
      stage_item<2>(acc + (int64_t)(f) * b.as + vc0, acc + (int64_t)(f) * b.as + vc1, wb, &GRF_BUF(bb)[(slot) * 64]); \
  } while (0)
#define GRF_PHASE_SYNC()                        \
  do {                                          \
    __builtin_amdgcn_sched_barrier(0);          \
    __builtin_amdgcn_s_waitcnt(kWaitAllVmLgkm); \
    __builtin_amdgcn_sched_barrier(0);          \
  } while (0)
#define GRF_P(n) P.n
#define GRF_RHS_ST(f, v, bb, sko, su0, sacc) \
  stage_one_st<MODE>(f, (v), GRF_LDS(bb, sko), GRF_LDS(bb, su0), GRF_LDS(bb, sacc), b, c, s, out, acc, sc, flags)
#define GRF_PIVCHK(v) bad |= !(fabs(v) <= 1e12)
#define GRF_SHIFT_ADVEC (SHIFTADV != 0)
#define GRF_STAGE_RHS_ONLY (MODE == 0)
  // nothing of an earlier call may still read the buffers or write memory
  GRF_PHASE_SYNC();
  if constexpr (VAR == 1) {
#include "gen/gen_rhs_staged_dec.inc"
  } else if constexpr (VAR == 2) {
#include "gen/gen_rhs_staged_lin.inc"
  } else {
#include "gen/gen_rhs_staged.inc"
  }
#undef GRF_STAGE_RHS_ONLY
#undef GRF_SHIFT_ADVEC
#undef GRF_PIVCHK
#undef GRF_RHS_ST
#undef GRF_P
#undef GRF_PHASE_SYNC
#undef GRF_STAGE_ACC
#undef GRF_STAGE_U0
#undef GRF_STAGE_U
#undef GRF_STAGE_KO
#undef GRF_STAGE_D
#undef GRF_LDS
#undef GRF_BUF
  if (bad) flags |= 2u;
  if (!(us[(int64_t)F_CHI * b.fs + s] > 0.0) || !(us[(int64_t)F_LAPSE * b.fs + s] > 0.0)) flags |= 4u;
  if (flags) atomicOr(status, flags);
}

// VAR 0: the full theory with the quadratic coupling; 1: the decoupling limit
// (the scalar does not source the metric); 2: the full theory with the
// general coupling (linear and exponential terms)
template <int MODE, int SHIFTADV, int VAR = 0>
__global__ __launch_bounds__(kStagedThreads) void k_point_staged(BoxDev b, grf_point_params P,
                                                                 const double* __restrict__ us,
                                                                 const double* __restrict__ D,
                                                                 const double* __restrict__ u0,
                                                                 double* __restrict__ out, double* __restrict__ acc,
                                                                 StageCoef sc, unsigned* __restrict__ status) {
  __shared__ double lbuf0_[GRF_STAGE_SLOTS * 64];
  __shared__ double lbuf1_[GRF_STAGE_SLOTS * 64];
  // the buffers as LDS-typed pointers, so that slot addresses are plain LDS
  // offsets (no generic-pointer conversion at each copy)
  staged_wave<MODE, SHIFTADV, VAR>(b, (int64_t)blockIdx.x * kStagedThreads, P, us, D, u0, out, acc, sc, status,
                                   (grf_lds_double*)lbuf0_, (grf_lds_double*)lbuf1_);
}

}  // namespace grf
