// libgrf: C-ABI entry points of the MI355X 4dST/CCZ4 right-hand side and RK4
// stage (declarations and argument conventions in include/grf.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/grf.h"
#include "kernels_fwd.h"
#include "kernels_vjp.h"
#include "kernels_batch.h"
#include "launch.h"

#include <map>
#include <mutex>
#include <tuple>

namespace grf {

thread_local std::string g_err;

grf_status fail(grf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define GRF_HIP_CHECK(call)                                                        \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) return fail(GRF_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kStatusBytes = 256;

grf_status check_box(const grf_box* b) {
  if (!b) return fail(GRF_EINVAL, "box is null");
  if (b->ng != 3 && b->ng != 4) return fail(GRF_ESHAPE, "ng must be 3 or 4 (got %d)", b->ng);
  if (b->nx < 1 || b->ny < 1 || b->nz < 1) return fail(GRF_ESHAPE, "box dims must be >= 1");
  const int e = 2 * b->ng;
  if ((int64_t)b->nx + e > (1 << 20) || (int64_t)b->ny + e > (1 << 20) || (int64_t)b->nz + e > (1 << 20))
    return fail(GRF_ESHAPE, "box too large");
  const int64_t need = (int64_t)(b->nx + e) * (b->ny + e) * (b->nz + e);
  if (b->field_stride < need) return fail(GRF_ESHAPE, "field_stride %lld < %lld", (long long)b->field_stride, (long long)need);
  if (!(b->dx > 0.0) || !(b->dy > 0.0) || !(b->dz > 0.0)) return fail(GRF_EINVAL, "spacing must be > 0");
  if (b->bc != GRF_BC_FROZEN && b->bc != GRF_BC_PERIODIC) return fail(GRF_EINVAL, "unknown bc %d", b->bc);
  return GRF_OK;
}

// entry points whose kernels assume three ghost layers
grf_status check_box3(const grf_box* b) {
  grf_status s = check_box(b);
  if (s != GRF_OK) return s;
  if (b->ng != 3)
    return fail(GRF_EUNSUPPORTED, "four ghost layers are not supported by the batched form");
  return GRF_OK;
}

grf_status check_params(const grf_params* p) {
  if (!p) return fail(GRF_EINVAL, "params is null");
  if (p->lambda_kind != GRF_LAMBDA_QUADRATIC) return fail(GRF_EUNSUPPORTED, "only lambda_kind 0 (quadratic)");
  if (p->lapse_power != 1.0) return fail(GRF_EUNSUPPORTED, "only lapse_power 1");
  if (p->a_gauge == -1.0 || p->b_gauge == -1.0) return fail(GRF_EINVAL, "a and b must differ from -1");
  if (p->enforce != 0 && p->enforce != 1) return fail(GRF_EINVAL, "enforce must be 0 or 1");
  if (p->decoupled != 0 && p->decoupled != 1) return fail(GRF_EINVAL, "decoupled must be 0 or 1");
  if (p->fd_order != 0 && p->fd_order != 4 && p->fd_order != 6) return fail(GRF_EINVAL, "fd_order must be 4 or 6");
  if (!std::isfinite(p->lambda_lin) || !std::isfinite(p->beta)) return fail(GRF_EINVAL, "lambda_lin/beta not finite");
  if (p->enforce && !(std::isfinite(p->chi_min) && std::isfinite(p->lapse_min)))
    return fail(GRF_EINVAL, "chi_min and lapse_min must be finite");
  return GRF_OK;
}

BoxDev make_boxdev(const grf_box* b) {
  BoxDev d;
  d.nx = b->nx;
  d.ny = b->ny;
  d.nz = b->nz;
  d.ng = b->ng;
  d.sy = b->nx + 2 * b->ng;
  d.sz = (int64_t)(b->nx + 2 * b->ng) * (b->ny + 2 * b->ng);
  d.fs = b->field_stride;
  d.ncell = (int64_t)b->nx * b->ny * b->nz;
  d.as = d.ncell;
  const double h[3] = {b->dx, b->dy, b->dz};
  for (int k = 0; k < 3; ++k) {
    d.i12h[k] = 1.0 / (12.0 * h[k]);
    d.i12h2[k] = 1.0 / (12.0 * h[k] * h[k]);
    d.i64h[k] = 1.0 / (64.0 * h[k]);
  }
  d.i144[0] = 1.0 / (144.0 * h[0] * h[1]);
  d.i144[1] = 1.0 / (144.0 * h[0] * h[2]);
  d.i144[2] = 1.0 / (144.0 * h[1] * h[2]);
  for (int k = 0; k < 3; ++k) {
    d.i60h[k] = 1.0 / (60.0 * h[k]);
    d.i180h2[k] = 1.0 / (180.0 * h[k] * h[k]);
  }
  d.i3600[0] = 1.0 / (3600.0 * h[0] * h[1]);
  d.i3600[1] = 1.0 / (3600.0 * h[0] * h[2]);
  d.i3600[2] = 1.0 / (3600.0 * h[1] * h[2]);
  for (int k = 0; k < 3; ++k) d.i256h[k] = 1.0 / (256.0 * h[k]);
  return d;
}

// The pointwise, enforcement and diagnostic kernels address interior cell
// (i, j, k) at (k+3) sz + (j+3) sy + (i+3) of the state they are given; on a
// box with four ghost layers they are given the state moved by one cell
// along each axis (same strides), which puts that address at (k+4, j+4, i+4).
int64_t interior_shift(const BoxDev& bd) { return (int64_t)(bd.ng - 3) * (bd.sz + bd.sy + 1); }

grf_point_params make_pp(const grf_params* p) {
  grf_point_params q;
  const double a = p->a_gauge, b = p->b_gauge, k1 = p->kappa1, k2 = p->kappa2;
  q.lambda_gb = p->lambda_gb;
  q.g2 = p->g2;
  q.kappa1 = k1;
  q.kappa3 = p->kappa3;
  q.k1_1pk2 = k1 * (1.0 + k2);
  q.k1_2pk2 = k1 * (2.0 + k2);
  q.k1k2 = k1 * k2;
  q.lapse_coeff = p->lapse_coeff;
  q.lapse_advec = p->lapse_advec;
  q.shift_gamma_coeff = p->shift_gamma_coeff;
  q.shift_advec = p->shift_advec;
  q.eta = p->eta;
  q.inv1pa = 1.0 / (1.0 + a);
  q.a_1pa = a / (1.0 + a);
  q.fb = b / (1.0 + b);
  q.cfac = 1.0 / (1.0 + b);
  q.b4 = b / (4.0 * (1.0 + b));
  q.lambda_lin = p->lambda_lin;
  q.beta = p->beta;
  return q;
}

// Stage path of the single-box calls, both a stencil kernel writing the
// record of the whole box and a pointwise kernel reading it: 0 = the plain
// pointwise kernel, 2 = the pointwise kernel with its inputs staged through
// LDS (the default).  The plain kernel carries the same algebra in another
// emission of the generated code (depth-first order, the general coupling),
// so the two check each other bit for bit.
int g_stage_path = 2;

size_t deriv_bytes(const grf_box* b) {
  return (size_t)GRF_NCOMP * (size_t)b->nx * b->ny * b->nz * sizeof(double);
}

constexpr int kTileVariantsMax = kDerivVariants;
// stencil variants the batched form can run (tiled shapes, z-marching 16x8x32, 32x8x32, 16x16x32)
constexpr int kBatchVariants[] = {0, 1, 2, 3, 4, 5, 6, 8};
int g_tile_variant = -1;  // -1: chosen per box (tile_variant_for)

// Stencil variant of a single-box call: the one grf_set_tile_variant chose, or
// by default the z-marching 128x8 column for boxes at least 128 cells wide and
// the 16x16 column for narrower ones (on a 64^3 box 0.148 ms per launch
// against 0.207 ms for the 128-wide column, half of whose threads have no
// cell there).
int tile_variant_for(const BoxDev& bd) {
  if (g_tile_variant >= 0) return g_tile_variant;
  return bd.nx >= 128 ? 9 : 8;
}

// Optional per-kernel timing with HIP events recorded on the launch stream
// around each stencil-stage and pointwise launch (enabled by grf_prof_begin).
struct ProfClass {
  std::vector<hipEvent_t> ev;  // start/end pairs
  int used = 0;
};
struct Prof {
  bool on = false;
  int cap = 0;
  ProfClass cls[4];  // 0 stencil stage, 1 pointwise/RK4, 2 VJP kernels, 3 the reverse pointwise kernel
} g_prof;

void prof_mark(int which, hipStream_t st) {
  if (!g_prof.on) return;
  ProfClass& c = g_prof.cls[which];
  if (c.used >= g_prof.cap * 2) return;
  hipEventRecord(c.ev[c.used++], st);
}

hipError_t launch_point(int mode, int sa, const BoxDev& bd, const grf_point_params& pp, const double* us,
                        const double* D, const double* u0, double* out, double* acc, StageCoef sc, unsigned* status,
                        hipStream_t st) {
  switch (mode) {
    case 1: return launch_point_m<1>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
    case 2: return launch_point_m<2>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
    case 4: return launch_point_m<4>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
    default: return launch_point_m<0>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
  }
}

hipError_t launch_staged(int mode, int sa, const BoxDev& bd, const grf_point_params& pp, const double* us,
                         const double* D, const double* u0, double* out, double* acc, StageCoef sc,
                         unsigned* status, hipStream_t st) {
  switch (mode) {
    case 1: return launch_staged_m<1>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
    case 2: return launch_staged_m<2>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
    case 4: return launch_staged_m<4>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
    default: return launch_staged_m<0>(sa, bd, pp, us, D, u0, out, acc, sc, status, st);
  }
}

// pointwise kernel of the split path: 0 plain, 2 with staged inputs
hipError_t launch_pointwise(int path, int mode, int sa, const BoxDev& bd, const grf_point_params& pp,
                            const double* us, const double* D, const double* u0, double* out, double* acc,
                            StageCoef sc, unsigned* status, hipStream_t st) {
  if (path == 2) return launch_staged(mode, sa, bd, pp, us, D, u0, out, acc, sc, status, st);
  // the plain kernel's code always carries the general coupling; only the
  // shift-advection bit selects its instance
  return launch_point(mode, sa & 1, bd, pp, us, D, u0, out, acc, sc, status, st);
}

hipError_t launch_point_batch(int mode, int sa, int grid, const BatchBoxDev* boxes, const CellEntry* cells,
                              int ncells, int stage, const grf_point_params& pp, unsigned* status,
                              hipStream_t st) {
  switch (mode) {
    case 1: return launch_point_batch_m<1>(sa, grid, boxes, cells, ncells, stage, pp, status, st);
    case 2: return launch_point_batch_m<2>(sa, grid, boxes, cells, ncells, stage, pp, status, st);
    default: return launch_point_batch_m<4>(sa, grid, boxes, cells, ncells, stage, pp, status, st);
  }
}

}  // namespace grf

using namespace grf;

extern "C" {

size_t grf_workspace_bytes(const grf_box* box) {
  if (check_box(box) != GRF_OK) return 0;
  return kStatusBytes + deriv_bytes(box);
}

const char* grf_last_error(void) { return g_err.c_str(); }

int64_t grf_flops_per_cell(int which) {
  switch (which) {
    case 0: return GRF_FLOPS_RHS;
    case 1: return GRF_FLOPS_RHS_SHIFTADV;
    case 2: return GRF_FLOPS_VJP;
    case 3: return GRF_FLOPS_CONSTRAINTS;
    case 4: return GRF_FLOPS_ENERGY;
    case 5: return GRF_FLOPS_RHS_DECOUPLED;
    case 6: return GRF_FLOPS_COUPLING;
    default: return -1;
  }
}

grf_status grf_status_clear(void* workspace, hipStream_t stream) {
  if (!workspace) return fail(GRF_EINVAL, "workspace is null");
  GRF_HIP_CHECK(launch_status_clear((unsigned*)workspace, stream));
  return GRF_OK;
}

grf_status grf_status_fetch(const void* workspace, hipStream_t stream, uint32_t* bits) {
  if (!workspace) return fail(GRF_EINVAL, "workspace is null");
  unsigned host = 0;
  GRF_HIP_CHECK(hipMemcpyAsync(&host, workspace, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
  GRF_HIP_CHECK(hipStreamSynchronize(stream));
  if (bits) *bits = host;
  if (host & GRF_FLAG_NONFINITE) return fail(GRF_ENONFINITE, "non-finite right-hand side");
  if (host & GRF_FLAG_HYPERBOLIC) return fail(GRF_EHYPERBOLIC, "near-singular per-cell system");
  if (host & GRF_FLAG_NONPOSITIVE) return fail(GRF_ENONPOSITIVE, "chi or lapse not positive");
  return GRF_OK;
}

grf_status grf_fill_periodic(const grf_box* box, double* u, hipStream_t stream) {
  grf_status s = check_box(box);
  if (s != GRF_OK) return s;
  if (!u) return fail(GRF_EINVAL, "u is null");
  BoxDev bd = make_boxdev(box);
  GRF_HIP_CHECK(launch_periodic(bd, u, stream));
  return GRF_OK;
}

static grf_status common_checks(const grf_params* p, const grf_box* box, void* ws, size_t ws_bytes) {
  grf_status s = check_params(p);
  if (s != GRF_OK) return s;
  s = check_box(box);
  if (s != GRF_OK) return s;
  if (box->ng == 4 && p->fd_order != 6) return fail(GRF_EUNSUPPORTED, "four ghost layers only with fd_order 6");
  if (!ws) return fail(GRF_EINVAL, "workspace is null");
  if (ws_bytes < kStatusBytes + deriv_bytes(box))
    return fail(GRF_ENOMEM, "workspace %zu bytes < %zu", ws_bytes, kStatusBytes + deriv_bytes(box));
  return GRF_OK;
}

// variant code of the staged pointwise kernel: bit 0 shift advection, then
// 2 the decoupling limit (its code carries the general coupling), 4 the full
// theory with the general coupling (linear and exponential terms; the
// default code has the quadratic coupling alone)
static int staged_variant(const grf_params* p, int sa) {
  if (p->decoupled) return sa | 2;
  return sa | (p->lambda_lin != 0.0 || p->beta != 0.0 ? 4 : 0);
}

// stencil stage of the forward paths at the parameters' finite-difference order
static hipError_t launch_deriv_p(const grf_params* p, const BoxDev& bd, const double* u, double* D, int sa,
                                 hipStream_t stream) {
  if (p->fd_order == 6) return launch_deriv6(bd, u, D, p->ko_sigma, sa, nullptr, stream);
  return launch_deriv(tile_variant_for(bd), bd, u, D, p->ko_sigma, sa, nullptr, stream);
}

// Interior planes per z-slab of the split stage paths: 0 = the whole box in
// one stencil launch and one pointwise launch (record of the whole box);
// n > 0 = slabs of n planes, each a stencil launch writing the slab's record
// and a pointwise launch reading it, so that the record held between the two
// is slab-sized.
static int g_slab_planes = 0;

// Stencil stage + pointwise stage (mode 0: right-hand side into out; 1, 2, 4:
// RK4 stage) of the split paths over z-slabs of at most `planes` interior
// planes.  Each slab is a sub-box: the state pointers move to its first plane
// (its ghost planes are the neighbouring planes of the box, or the box's own
// ghosts at the ends), its record in D is compact over the slab, and the
// accumulator keeps the whole box's field stride.  Per cell the arithmetic is
// that of the whole-box launches, so results are bitwise identical.
// path: the stage path (0 or 2), read once by the caller.
static hipError_t split_stage(const grf_params* p, const BoxDev& bd, int path, int planes, int mode, StageCoef sc,
                              const double* us, const double* u0, double* out, double* acc, double* D,
                              unsigned* status, hipStream_t stream) {
  const grf_point_params pp = make_pp(p);
  const int sa = p->shift_advec != 0.0;
  const int var = staged_variant(p, sa);
  const int64_t sh = interior_shift(bd);
  const int64_t plane = (int64_t)bd.nx * bd.ny;
  if (planes <= 0 || planes > bd.nz) planes = bd.nz;
  for (int z0 = 0; z0 < bd.nz; z0 += planes) {
    BoxDev sb = bd;
    sb.nz = planes < bd.nz - z0 ? planes : bd.nz - z0;
    sb.ncell = plane * sb.nz;
    sb.as = bd.ncell;
    const int64_t so = (int64_t)z0 * bd.sz;
    prof_mark(0, stream);
    hipError_t e = launch_deriv_p(p, sb, us + so, D, sa, stream);
    if (e != hipSuccess) return e;
    prof_mark(0, stream);
    prof_mark(1, stream);
    e = launch_pointwise(path, mode, var, sb, pp, us + so + sh, D, u0 ? u0 + so + sh : nullptr, out + so + sh,
                         acc ? acc + (int64_t)z0 * plane : nullptr, sc, status, stream);
    if (e != hipSuccess) return e;
    prof_mark(1, stream);
  }
  return hipSuccess;
}

grf_status grf_rhs_eval(const grf_params* p, const grf_box* box, const double* u, double* rhs, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
  grf_status s = common_checks(p, box, workspace, workspace_bytes);
  if (s != GRF_OK) return s;
  if (!u || !rhs) return fail(GRF_EINVAL, "u/rhs is null");
  if (u == rhs) return fail(GRF_EINVAL, "rhs must not alias u");
  BoxDev bd = make_boxdev(box);
  unsigned* status = (unsigned*)workspace;
  double* D = (double*)((char*)workspace + kStatusBytes);
  const int path = g_stage_path;
  if (p->decoupled && path != 2)
    return fail(GRF_EUNSUPPORTED, "the decoupling limit runs on stage path 2 only");
  GRF_HIP_CHECK(split_stage(p, bd, path, g_slab_planes, 0, StageCoef{0.0}, u, nullptr, rhs, nullptr, D, status,
                            stream));
  return GRF_OK;
}

static grf_status rk4_stage_impl(const grf_params* p, const grf_box* box, int stage, double dt, const double* u0,
                                 const double* us, double* unext, double* acc, void* workspace,
                                 size_t workspace_bytes, hipStream_t stream, bool box_ghosts);

grf_status grf_rk4_stage(const grf_params* p, const grf_box* box, int stage, double dt, const double* u0,
                         const double* us, double* unext, double* acc, void* workspace, size_t workspace_bytes,
                         hipStream_t stream) {
  return rk4_stage_impl(p, box, stage, dt, u0, us, unext, acc, workspace, workspace_bytes, stream, true);
}

// interior stage; box_ghosts: apply the box's own ghost rule (periodic fill)
static grf_status rk4_stage_impl(const grf_params* p, const grf_box* box, int stage, double dt, const double* u0,
                                 const double* us, double* unext, double* acc, void* workspace,
                                 size_t workspace_bytes, hipStream_t stream, bool box_ghosts) {
  grf_status s = common_checks(p, box, workspace, workspace_bytes);
  if (s != GRF_OK) return s;
  if (stage < 1 || stage > 4) return fail(GRF_EINVAL, "stage must be 1..4 (got %d)", stage);
  if (!u0 || !us || !unext || !acc) return fail(GRF_EINVAL, "null state pointer");
  if (unext == us || unext == u0) return fail(GRF_EINVAL, "unext must not alias us or u0");
  if (!std::isfinite(dt)) return fail(GRF_EINVAL, "dt not finite");
  BoxDev bd = make_boxdev(box);
  unsigned* status = (unsigned*)workspace;
  double* D = (double*)((char*)workspace + kStatusBytes);
  const int path = g_stage_path;
  if (p->decoupled && path != 2)
    return fail(GRF_EUNSUPPORTED, "the decoupling limit runs on stage path 2 only");
  StageCoef sc;
  int mode;
  switch (stage) {
    case 1: mode = 1; sc = StageCoef{0.5 * dt}; break;
    case 2: mode = 2; sc = StageCoef{0.5 * dt}; break;
    case 3: mode = 2; sc = StageCoef{1.0 * dt}; break;
    default: mode = 4; sc = StageCoef{dt / 6.0}; break;
  }
  GRF_HIP_CHECK(split_stage(p, bd, path, g_slab_planes, mode, sc, us, u0, unext, acc, D, status, stream));
  if (p->enforce)
    GRF_HIP_CHECK(launch_enforce(bd, unext + interior_shift(bd), p->chi_min, p->lapse_min, stream));
  if (box_ghosts && box->bc == GRF_BC_PERIODIC) GRF_HIP_CHECK(launch_periodic(bd, unext, stream));
  return GRF_OK;
}

// ---- RK4 stage without allocation or workspace
//
// The derivative records of grf_rk4_stage_static live in this file-scope
// device array, one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only stands for the
// symbol); its device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the current device's copy).
static grf_status static_scratch(double** out) {
  int dev = -1;
  GRF_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GRF_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    GRF_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(GRF_EHIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = (double*)g_scratch_ptr[dev];
  return GRF_OK;
}

extern "C" grf_status grf_rk4_stage_static(const grf_params* p, const grf_box* box, int stage, double dt,
                                           const double* u0, const double* us, double* unext, double* acc,
                                           uint32_t* status, hipStream_t stream) {
  grf_status s = check_params(p);
  if (s != GRF_OK) return s;
  s = check_box(box);
  if (s != GRF_OK) return s;
  if (box->ng == 4 && p->fd_order != 6) return fail(GRF_EUNSUPPORTED, "four ghost layers only with fd_order 6");
  if (stage < 1 || stage > 4) return fail(GRF_EINVAL, "stage must be 1..4 (got %d)", stage);
  if (!u0 || !us || !unext || !acc || !status) return fail(GRF_EINVAL, "null pointer argument");
  if (unext == us || unext == u0) return fail(GRF_EINVAL, "unext must not alias us or u0");
  if (!std::isfinite(dt)) return fail(GRF_EINVAL, "dt not finite");
  const int64_t plane = (int64_t)box->nx * box->ny;
  const int64_t cap = (int64_t)(kStaticScratchBytes / (GRF_NCOMP * sizeof(double)));
  if (plane > cap)
    return fail(GRF_ENOMEM, "one z-plane of %lld cells exceeds the static scratch (%lld cells, %zu bytes)",
                (long long)plane, (long long)cap, kStaticScratchBytes);
  double* D = nullptr;
  s = static_scratch(&D);
  if (s != GRF_OK) return s;
  BoxDev bd = make_boxdev(box);
  int planes = (int)(cap / plane < box->nz ? cap / plane : box->nz);
  if (g_slab_planes > 0 && g_slab_planes < planes) planes = g_slab_planes;
  StageCoef sc;
  int mode;
  switch (stage) {
    case 1: mode = 1; sc = StageCoef{0.5 * dt}; break;
    case 2: mode = 2; sc = StageCoef{0.5 * dt}; break;
    case 3: mode = 2; sc = StageCoef{1.0 * dt}; break;
    default: mode = 4; sc = StageCoef{dt / 6.0}; break;
  }
  // the split path with staged pointwise inputs, whatever grf_set_stage_path chose
  const hipError_t e = split_stage(p, bd, 2, planes, mode, sc, us, u0, unext, acc, D, (unsigned*)status, stream);
  if (e != hipSuccess) return fail(GRF_EHIP, "grf_rk4_stage_static: %s", hipGetErrorString(e));
  if (p->enforce)
    GRF_HIP_CHECK(launch_enforce(bd, unext + interior_shift(bd), p->chi_min, p->lapse_min, stream));
  if (box->bc == GRF_BC_PERIODIC) GRF_HIP_CHECK(launch_periodic(bd, unext, stream));
  return GRF_OK;
}

// ---- per-face boundary rules

// tensor indices of each field along each axis (reflection sign = (-1)^count)
static int index_count(int f, int axis) {
  static const int sym[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};  // h_ij / A_ij packing
  if (f >= 1 && f <= 6) return (sym[f - 1][0] == axis) + (sym[f - 1][1] == axis);    // h_ij
  if (f >= 8 && f <= 13) return (sym[f - 8][0] == axis) + (sym[f - 8][1] == axis);   // A_ij
  if (f >= 15 && f <= 17) return f - 15 == axis;                                     // Gamma^i
  if (f >= 19 && f <= 21) return f - 19 == axis;                                     // beta^i
  if (f >= 22 && f <= 24) return f - 22 == axis;                                     // B^i
  return 0;
}

static grf_status make_bcdev(const grf_bc* bc, const grf_box* box, bool radiative, BcDev& d) {
  if (!bc) return fail(GRF_EINVAL, "bc is null");
  const int n[3] = {box->nx, box->ny, box->nz};
  const double h[3] = {box->dx, box->dy, box->dz};
  for (int f = 0; f < 6; ++f) {
    const int r = bc->rule[f];
    if (r < GRF_FACE_FROZEN || r > GRF_FACE_SOMMERFELD) return fail(GRF_EINVAL, "face %d: unknown rule %d", f, r);
    const int axis = f / 2;
    if (r == GRF_FACE_PERIODIC && bc->rule[f ^ 1] != GRF_FACE_PERIODIC)
      return fail(GRF_EINVAL, "face %d: periodic faces come in pairs", f);
    if (r == GRF_FACE_REFLECTIVE && n[axis] < box->ng)
      return fail(GRF_EINVAL, "face %d: reflective needs >= %d cells (the ghost count)", f, box->ng);
    if (r == GRF_FACE_EXTRAPOLATING && bc->extrap_order == 1 && n[axis] < 2)
      return fail(GRF_EINVAL, "face %d: linear extrapolation needs >= 2 cells", f);
    d.rule[f] = r;
  }
  if (bc->extrap_order != 0 && bc->extrap_order != 1) return fail(GRF_EINVAL, "extrap_order must be 0 or 1");
  if (bc->parity_phi != 1 && bc->parity_phi != -1) return fail(GRF_EINVAL, "parity_phi must be +1 or -1");
  d.extrap_order = bc->extrap_order;
  const double origin[3] = {box->x0, box->y0, box->z0};
  for (int a = 0; a < 3; ++a) {
    d.origin[a] = origin[a];
    d.centre[a] = bc->centre[a];
    d.h[a] = h[a];
    d.i2h[a] = 1.0 / (2.0 * h[a]);
    for (int f = 0; f < NF; ++f)
      d.sign[a][f] = (f == 25 || f == 26) ? (double)bc->parity_phi : ((index_count(f, a) & 1) ? -1.0 : 1.0);
  }
  for (int f = 0; f < NF; ++f) {
    d.speed[f] = bc->speed[f];
    d.asymptote[f] = bc->asymptote[f];
  }
  bool somm = false;
  for (int f = 0; f < 6; ++f) somm |= d.rule[f] == GRF_FACE_SOMMERFELD;
  if (radiative && somm) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(origin[a]) || !std::isfinite(bc->centre[a])) return fail(GRF_EINVAL, "origin/centre not finite");
    for (int f = 0; f < NF; ++f)
      if (!std::isfinite(bc->speed[f]) || !std::isfinite(bc->asymptote[f]))
        return fail(GRF_EINVAL, "speed/asymptote of field %d not finite", f);
    // the centre must not coincide with a ghost cell centre (r = 0 there)
    bool on_cell = true, ghost = false;
    for (int a = 0; a < 3; ++a) {
      const double t = (bc->centre[a] - origin[a]) / h[a];
      const double m = std::nearbyint(t);
      on_cell &= std::fabs(t - m) < 1e-9 && m >= -(double)box->ng && m <= n[a] + box->ng - 1.0;
      ghost |= m < 0.0 || m >= n[a];
    }
    if (on_cell && ghost) return fail(GRF_EINVAL, "the radiative centre is a ghost cell centre");
  }
  return GRF_OK;
}

int64_t grf_bc_ghost_cells(const grf_box* box) {
  if (check_box(box) != GRF_OK) return 0;
  return ghost_cells(make_boxdev(box));
}

grf_status grf_bc_fill(const grf_bc* bc, const grf_box* box, double* u, hipStream_t stream) {
  grf_status s = check_box(box);
  if (s != GRF_OK) return s;
  if (!u) return fail(GRF_EINVAL, "u is null");
  BcDev d;
  if ((s = make_bcdev(bc, box, false, d)) != GRF_OK) return s;
  GRF_HIP_CHECK(launch_bc_fill(make_boxdev(box), d, u, stream));
  return GRF_OK;
}

grf_status grf_bc_ghost_rhs(const grf_bc* bc, const grf_box* box, const double* u, double* rhs,
                            hipStream_t stream) {
  grf_status s = check_box(box);
  if (s != GRF_OK) return s;
  if (!u || !rhs) return fail(GRF_EINVAL, "u/rhs is null");
  if (u == rhs) return fail(GRF_EINVAL, "rhs must not alias u");
  BcDev d;
  if ((s = make_bcdev(bc, box, true, d)) != GRF_OK) return s;
  GRF_HIP_CHECK(launch_bc_ghost(0, make_boxdev(box), d, u, nullptr, rhs, nullptr, StageCoef{0.0}, stream));
  return GRF_OK;
}

grf_status grf_rk4_stage_bc(const grf_params* p, const grf_box* box, const grf_bc* bc, int stage, double dt,
                            const double* u0, const double* us, double* unext, double* acc, double* gacc,
                            void* workspace, size_t workspace_bytes, hipStream_t stream) {
  grf_status s = check_box(box);
  if (s != GRF_OK) return s;
  BcDev d;
  if ((s = make_bcdev(bc, box, true, d)) != GRF_OK) return s;
  bool somm = false, fill = false;
  for (int f = 0; f < 6; ++f) {
    somm |= d.rule[f] == GRF_FACE_SOMMERFELD;
    fill |= d.rule[f] == GRF_FACE_PERIODIC || d.rule[f] == GRF_FACE_REFLECTIVE || d.rule[f] == GRF_FACE_EXTRAPOLATING;
  }
  if (somm && !gacc) return fail(GRF_EINVAL, "gacc is null");
  s = rk4_stage_impl(p, box, stage, dt, u0, us, unext, acc, workspace, workspace_bytes, stream, false);
  if (s != GRF_OK) return s;
  const BoxDev bd = make_boxdev(box);
  if (somm) {
    int mode;
    StageCoef sc;
    switch (stage) {
      case 1: mode = 1; sc = StageCoef{0.5 * dt}; break;
      case 2: mode = 2; sc = StageCoef{0.5 * dt}; break;
      case 3: mode = 2; sc = StageCoef{1.0 * dt}; break;
      default: mode = 4; sc = StageCoef{dt / 6.0}; break;
    }
    GRF_HIP_CHECK(launch_bc_ghost(mode, bd, d, us, u0, unext, gacc, sc, stream));
  }
  if (fill) GRF_HIP_CHECK(launch_bc_fill(bd, d, unext, stream));
  return GRF_OK;
}

static grf_status diagnostics(int which, const grf_params* p, const grf_box* box, const double* u, double* out,
                              void* workspace, size_t workspace_bytes, hipStream_t stream) {
  grf_status s = common_checks(p, box, workspace, workspace_bytes);
  if (s != GRF_OK) return s;
  if (!u || !out) return fail(GRF_EINVAL, "u/out is null");
  if (p->decoupled && which != 0)
    return fail(GRF_EUNSUPPORTED, "in the decoupling limit only the constraints are implemented");
  BoxDev bd = make_boxdev(box);
  grf_point_params pp = make_pp(p);
  double* D = (double*)((char*)workspace + kStatusBytes);
  GRF_HIP_CHECK(launch_deriv_p(p, bd, u, D, p->shift_advec != 0.0, stream));
  GRF_HIP_CHECK(launch_constraints(p->decoupled ? 3 : which, bd, pp, u + interior_shift(bd), D, out, stream));
  return GRF_OK;
}

grf_status grf_constraints(const grf_params* p, const grf_box* box, const double* u, double* out, void* workspace,
                           size_t workspace_bytes, hipStream_t stream) {
  return diagnostics(0, p, box, u, out, workspace, workspace_bytes, stream);
}

grf_status grf_energy_densities(const grf_params* p, const grf_box* box, const double* u, double* out,
                                void* workspace, size_t workspace_bytes, hipStream_t stream) {
  return diagnostics(1, p, box, u, out, workspace, workspace_bytes, stream);
}

grf_status grf_coupling_diagnostics(const grf_params* p, const grf_box* box, const double* u, double* out,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream) {
  return diagnostics(2, p, box, u, out, workspace, workspace_bytes, stream);
}

grf_status grf_enforce(const grf_params* p, const grf_box* box, double* u, hipStream_t stream) {
  grf_status s = check_params(p);
  if (s != GRF_OK) return s;
  if ((s = check_box(box)) != GRF_OK) return s;
  if (!u) return fail(GRF_EINVAL, "u is null");
  BoxDev bd = make_boxdev(box);
  GRF_HIP_CHECK(launch_enforce(bd, u + interior_shift(bd), p->chi_min, p->lapse_min, stream));
  return GRF_OK;
}

}  // extern "C"

namespace grf {
constexpr int64_t kRedChunk = 4096;
struct VjpLayout {
  size_t off_D, off_UP, off_Dbar, off_TH, off_part, total;
  int nparts;
};
VjpLayout vjp_layout(const grf_box* b) {
  const size_t n = (size_t)b->nx * b->ny * b->nz;
  VjpLayout L;
  L.nparts = (int)((n + kRedChunk - 1) / kRedChunk);
  L.off_D = kStatusBytes;
  L.off_UP = L.off_D + (size_t)GRF_NCOMP * n * 8;
  L.off_Dbar = L.off_UP + (size_t)3 * NF * n * 8;
  L.off_TH = L.off_Dbar + (size_t)NCOMP_BAR * n * 8;
  L.off_part = L.off_TH + (size_t)NTH * n * 8;
  L.total = L.off_part + (size_t)NTH * L.nparts * 8;
  return L;
}
}  // namespace grf

extern "C" {

size_t grf_vjp_workspace_bytes(const grf_box* box) {
  if (check_box(box) != GRF_OK) return 0;
  return vjp_layout(box).total;
}

grf_status grf_rhs_vjp(const grf_params* p, const grf_box* box, const double* u, const double* w, double* u_bar,
                       double* theta_bar, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  grf_status s = check_params(p);
  if (s != GRF_OK) return s;
  s = check_box(box);
  if (s != GRF_OK) return s;
  if (!u || !w || !u_bar || !theta_bar || !workspace) return fail(GRF_EINVAL, "null pointer");
  if (box->ng == 4 && p->fd_order != 6) return fail(GRF_EUNSUPPORTED, "four ghost layers only with fd_order 6");
  if (u_bar == u || u_bar == w) return fail(GRF_EINVAL, "u_bar must not alias u or w");
  if (p->lambda_lin != 0.0 || p->beta != 0.0)
    return fail(GRF_EUNSUPPORTED, "the adjoint takes the quadratic coupling (lambda_lin = beta = 0)");
  const VjpLayout L = vjp_layout(box);
  if (workspace_bytes < L.total) return fail(GRF_ENOMEM, "workspace %zu bytes < %zu", workspace_bytes, L.total);
  BoxDev bd = make_boxdev(box);
  grf_point_params pp = make_pp(p);
  char* ws = (char*)workspace;
  double* D = (double*)(ws + L.off_D);
  double* UP = (double*)(ws + L.off_UP);
  double* Dbar = (double*)(ws + L.off_Dbar);
  double* TH = (double*)(ws + L.off_TH);
  double* part = (double*)(ws + L.off_part);
  const int sa = p->shift_advec != 0.0;
  prof_mark(2, stream);
  const int order = p->fd_order == 6 ? 6 : 4;
  if (order == 6)
    GRF_HIP_CHECK(launch_deriv6(bd, u, D, p->ko_sigma, sa, UP, stream));
  else
    GRF_HIP_CHECK(launch_deriv(tile_variant_for(bd), bd, u, D, p->ko_sigma, sa, UP, stream));
  const int64_t sh = interior_shift(bd);
  if (p->decoupled)
    GRF_HIP_CHECK(launch_vjp_point_dec(sa, bd, pp, u + sh, D, UP, w + sh, u_bar + sh, Dbar, TH, stream));
  else
  {
    prof_mark(3, stream);
    GRF_HIP_CHECK(launch_vjp_point(sa, bd, pp, u + sh, D, UP, w + sh, u_bar + sh, Dbar, TH, stream));
    prof_mark(3, stream);
  }
  GRF_HIP_CHECK(launch_vjp_transpose(bd, u, w, Dbar, p->ko_sigma, sa, order, u_bar, stream));
  GRF_HIP_CHECK(launch_reduce(TH, bd.ncell, kRedChunk, L.nparts, part, theta_bar, stream));
  prof_mark(2, stream);
  return GRF_OK;
}

size_t grf_rk4_step_vjp_workspace_bytes(const grf_box* box) {
  if (check_box(box) != GRF_OK) return 0;
  const size_t state = (size_t)NF * box->field_stride * 8;
  return vjp_layout(box).total + 2 * ((state + 255) / 256 * 256);
}

grf_status grf_rk4_step_vjp(const grf_params* p, const grf_box* box, double dt, const double* u, const double* u2,
                            const double* u3, const double* u4, const double* ubar_new, double* ubar,
                            double* theta_bar, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  grf_status s = check_params(p);
  if (s != GRF_OK) return s;
  s = check_box(box);
  if (s != GRF_OK) return s;
  if (box->bc != GRF_BC_FROZEN) return fail(GRF_EUNSUPPORTED, "the step adjoint is implemented for frozen ghosts");
  if (box->ng == 4 && p->fd_order != 6) return fail(GRF_EUNSUPPORTED, "four ghost layers only with fd_order 6");
  if (p->enforce) return fail(GRF_EUNSUPPORTED, "the step adjoint does not differentiate the enforcement");
  if (p->lambda_lin != 0.0 || p->beta != 0.0)
    return fail(GRF_EUNSUPPORTED, "the adjoint takes the quadratic coupling (lambda_lin = beta = 0)");
  if (!u || !u2 || !u3 || !u4 || !ubar_new || !ubar || !theta_bar || !workspace) return fail(GRF_EINVAL, "null pointer");
  if (ubar == ubar_new || ubar == u || ubar == u2 || ubar == u3 || ubar == u4)
    return fail(GRF_EINVAL, "ubar must not alias an input");
  if (!std::isfinite(dt)) return fail(GRF_EINVAL, "dt not finite");
  const size_t need = grf_rk4_step_vjp_workspace_bytes(box);
  if (workspace_bytes < need) return fail(GRF_ENOMEM, "workspace %zu bytes < %zu", workspace_bytes, need);
  const VjpLayout L = vjp_layout(box);
  const size_t state = (size_t)NF * box->field_stride * 8;
  const size_t sstate = (state + 255) / 256 * 256;
  double* kbar = (double*)((char*)workspace + L.total);
  double* sbar = (double*)((char*)workspace + L.total + sstate);
  const int64_t n = (int64_t)NF * box->field_stride;
  auto vjp = [&](const double* at, const double* w, double* out) {
    return grf_rhs_vjp(p, box, at, w, out, theta_bar, workspace, L.total, stream);
  };
  // stage 4: k4 = f(u4), u_new = u + dt/6 (k1 + 2k2 + 2k3 + k4), u4 = u + dt k3
  GRF_HIP_CHECK(launch_axpby(n, dt / 6.0, ubar_new, 0.0, (const double*)nullptr, kbar, stream));
  GRF_HIP_CHECK(launch_fill(n, 0.0, sbar, stream));
  GRF_HIP_CHECK(hipGetLastError());
  if ((s = vjp(u4, kbar, sbar)) != GRF_OK) return s;
  GRF_HIP_CHECK(launch_axpby(n, 1.0, ubar_new, 1.0, (const double*)sbar, ubar, stream));
  // stage 3: k3 = f(u3), u3 = u + dt/2 k2
  GRF_HIP_CHECK(launch_axpby(n, dt / 3.0, ubar_new, dt, (const double*)sbar, kbar, stream));
  GRF_HIP_CHECK(launch_fill(n, 0.0, sbar, stream));
  GRF_HIP_CHECK(hipGetLastError());
  if ((s = vjp(u3, kbar, sbar)) != GRF_OK) return s;
  GRF_HIP_CHECK(launch_axpby(n, 1.0, (const double*)ubar, 1.0, (const double*)sbar, ubar, stream));
  // stage 2: k2 = f(u2), u2 = u + dt/2 k1
  GRF_HIP_CHECK(launch_axpby(n, dt / 3.0, ubar_new, 0.5 * dt, (const double*)sbar, kbar, stream));
  GRF_HIP_CHECK(launch_fill(n, 0.0, sbar, stream));
  GRF_HIP_CHECK(hipGetLastError());
  if ((s = vjp(u2, kbar, sbar)) != GRF_OK) return s;
  GRF_HIP_CHECK(launch_axpby(n, 1.0, (const double*)ubar, 1.0, (const double*)sbar, ubar, stream));
  // stage 1: k1 = f(u)
  GRF_HIP_CHECK(launch_axpby(n, dt / 6.0, ubar_new, 0.5 * dt, (const double*)sbar, kbar, stream));
  GRF_HIP_CHECK(hipGetLastError());
  if ((s = vjp(u, kbar, ubar)) != GRF_OK) return s;
  return GRF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched boxes
struct grf_batch {
  grf_params params;
  std::vector<grf_box> boxes;
  std::vector<grf::BatchBoxDev> host;  // descriptors (host copy)
  grf::BatchBoxDev* dev = nullptr;     // descriptors (device)
  std::vector<int> variant;            // stencil tile variant per box
  grf::TileEntry* tiles[grf::kTileVariantsMax] = {};
  int ntiles[grf::kTileVariantsMax] = {};
  grf::CellEntry* cells = nullptr;
  int ncells = 0;
  unsigned* status = nullptr;
  int grid_deriv[grf::kTileVariantsMax] = {};
  int grid_point = 0;
};

namespace grf {

std::map<std::tuple<int, int, int>, int> g_tile_cache;  // autotuned tile variant per box shape

// Cells an entry's workgroup stages (its tile or column chunk with the halo):
// the stencil stage's cost of the entry.
static int64_t entry_cost(int v, const BoxDev& bd, int t) {
  static const int shape[kTileVariantsMax][3] = {{16, 8, 4}, {32, 4, 4}, {8, 8, 8},  {16, 16, 2}, {64, 4, 2},
                                                 {16, 8, 32}, {32, 8, 32}, {32, 4, 32}, {16, 16, 32}, {128, 8, 32}};
  const int TX = shape[v][0], TY = shape[v][1], TZ = shape[v][2];
  const int ntx = (bd.nx + TX - 1) / TX, nty = (bd.ny + TY - 1) / TY;
  const int x0 = (t % ntx) * TX, y0 = (t / ntx % nty) * TY, z0 = (t / ntx / nty) * TZ;
  return (int64_t)(std::min(TX, bd.nx - x0) + 6) * (std::min(TY, bd.ny - y0) + 6) * (std::min(TZ, bd.nz - z0) + 6);
}

grf_status batch_upload_tiles(grf_batch* B) {
  std::vector<TileEntry> lists[kTileVariantsMax];
  for (size_t b = 0; b < B->boxes.size(); ++b) {
    const int v = B->variant[b];
    const int nt = tiles_of_variant(v, B->host[b].bd);
    for (int t = 0; t < nt; ++t) lists[v].push_back(TileEntry{(int)b, t});
  }
  // heaviest entries first: workgroups are dispatched in list order, so the
  // last ones to run are the light ones
  for (int v : kBatchVariants)
    std::stable_sort(lists[v].begin(), lists[v].end(), [&](const TileEntry& a, const TileEntry& c) {
      return entry_cost(v, B->host[a.box].bd, a.tile) > entry_cost(v, B->host[c.box].bd, c.tile);
    });
  for (int v : kBatchVariants) {
    if (B->tiles[v]) GRF_HIP_CHECK(hipFree(B->tiles[v]));
    B->tiles[v] = nullptr;
    B->ntiles[v] = (int)lists[v].size();
    if (lists[v].empty()) continue;
    GRF_HIP_CHECK(hipMalloc(&B->tiles[v], lists[v].size() * sizeof(TileEntry)));
    GRF_HIP_CHECK(hipMemcpy(B->tiles[v], lists[v].data(), lists[v].size() * sizeof(TileEntry), hipMemcpyHostToDevice));
    B->grid_deriv[v] = grid_deriv_batch(v, (int64_t)lists[v].size() * NF);
  }
  return GRF_OK;
}

grf_status batch_stage(grf_batch* B, int stage, hipStream_t st) {
  for (int v : kBatchVariants) {
    if (!B->ntiles[v]) continue;
    prof_mark(0, st);
    GRF_HIP_CHECK(launch_deriv_batch(v, B->grid_deriv[v], B->dev, B->tiles[v], B->ntiles[v], stage,
                                     B->params.ko_sigma, B->params.shift_advec != 0.0, st));
    prof_mark(0, st);
  }
  const grf_point_params pp = make_pp(&B->params);
  prof_mark(1, st);
  const int mode = stage == 1 ? 1 : (stage == 4 ? 4 : 2);
  GRF_HIP_CHECK(launch_point_batch(mode, B->params.shift_advec != 0.0, B->grid_point, B->dev, B->cells, B->ncells,
                                   stage, pp, B->status, st));
  prof_mark(1, st);
  return GRF_OK;
}

}  // namespace grf

extern "C" {

size_t grf_batch_scratch_bytes(const grf_box* boxes, int nboxes) {
  if (!boxes || nboxes < 1) return 0;
  size_t tot = 0;
  for (int b = 0; b < nboxes; ++b) {
    if (check_box3(&boxes[b]) != GRF_OK) return 0;
    const size_t n = (size_t)boxes[b].nx * boxes[b].ny * boxes[b].nz;
    const size_t state = (size_t)NF * boxes[b].field_stride * 8;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    tot += 2 * al(state) + al((size_t)NF * n * 8) + al((size_t)GRF_NCOMP * n * 8);
  }
  return tot;
}

grf_status grf_batch_create(const grf_params* p, const grf_box* boxes, int nboxes, double* const* u,
                            const double* dts, void* scratch, size_t scratch_bytes, grf_batch** out) {
  grf_status s = check_params(p);
  if (s != GRF_OK) return s;
  if (p->enforce) return fail(GRF_EUNSUPPORTED, "the batched form has no post-stage enforcement");
  if (p->decoupled) return fail(GRF_EUNSUPPORTED, "the batched form runs the full theory only");
  if (p->lambda_lin != 0.0 || p->beta != 0.0)
    return fail(GRF_EUNSUPPORTED, "the batched form has the quadratic coupling only");
  if (p->fd_order == 6) return fail(GRF_EUNSUPPORTED, "the batched form uses the fourth-order stencils only");
  if (!boxes || nboxes < 1 || !u || !dts || !out || !scratch) return fail(GRF_EINVAL, "null argument");
  for (int b = 0; b < nboxes; ++b) {
    if ((s = check_box3(&boxes[b])) != GRF_OK) return s;
    if (boxes[b].bc != GRF_BC_FROZEN) return fail(GRF_EUNSUPPORTED, "batched boxes use frozen ghosts");
    if (!u[b]) return fail(GRF_EINVAL, "null state of box %d", b);
    if (!std::isfinite(dts[b])) return fail(GRF_EINVAL, "dt of box %d not finite", b);
  }
  if (scratch_bytes < grf_batch_scratch_bytes(boxes, nboxes)) return fail(GRF_ENOMEM, "scratch too small");
  grf_batch* B = new grf_batch();
  B->params = *p;
  B->boxes.assign(boxes, boxes + nboxes);
  B->variant.assign(nboxes, 8);  // z-marching until autotuned
  char* sp = (char*)scratch;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  std::vector<CellEntry> cells;
  for (int b = 0; b < nboxes; ++b) {
    BatchBoxDev d;
    d.bd = make_boxdev(&boxes[b]);
    const size_t n = (size_t)d.bd.ncell;
    const size_t state = (size_t)NF * boxes[b].field_stride * 8;
    d.u = u[b];
    d.ub = (double*)sp; sp += al(state);
    d.ua = (double*)sp; sp += al(state);
    d.acc = (double*)sp; sp += al((size_t)NF * n * 8);
    d.D = (double*)sp; sp += al((size_t)GRF_NCOMP * n * 8);
    d.dt = dts[b];
    // the stage buffers carry the frozen ghosts of the initial state
    if (hipMemcpy(d.ub, d.u, state, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(d.ua, d.u, state, hipMemcpyDeviceToDevice) != hipSuccess) {
      delete B;
      return fail(GRF_EHIP, "initial copy of box %d failed", b);
    }
    B->host.push_back(d);
    const auto it = g_tile_cache.find(std::make_tuple(boxes[b].nx, boxes[b].ny, boxes[b].nz));
    if (it != g_tile_cache.end()) B->variant[b] = it->second;
    for (int64_t c0 = 0; c0 < (int64_t)n; c0 += kStagedThreads) cells.push_back(CellEntry{b, 0, c0});
  }
  auto cleanup = [&](grf_status code) {
    grf_batch_destroy(B);
    return code;
  };
  if (hipMalloc(&B->dev, nboxes * sizeof(BatchBoxDev)) != hipSuccess) return cleanup(fail(GRF_EHIP, "hipMalloc"));
  if (hipMemcpy(B->dev, B->host.data(), nboxes * sizeof(BatchBoxDev), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(GRF_EHIP, "hipMemcpy"));
  B->ncells = (int)cells.size();
  if (hipMalloc(&B->cells, cells.size() * sizeof(CellEntry)) != hipSuccess) return cleanup(fail(GRF_EHIP, "hipMalloc"));
  if (hipMemcpy(B->cells, cells.data(), cells.size() * sizeof(CellEntry), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(GRF_EHIP, "hipMemcpy"));
  if (hipMalloc(&B->status, 256) != hipSuccess) return cleanup(fail(GRF_EHIP, "hipMalloc"));
  if (hipMemset(B->status, 0, 256) != hipSuccess) return cleanup(fail(GRF_EHIP, "hipMemset"));
  B->grid_point = grid_point_batch_m<2>(p->shift_advec != 0.0, B->ncells);
  if ((s = batch_upload_tiles(B)) != GRF_OK) return cleanup(s);
  *out = B;
  return GRF_OK;
}

void grf_batch_destroy(grf_batch* B) {
  if (!B) return;
  if (B->dev) (void)hipFree(B->dev);
  if (B->cells) (void)hipFree(B->cells);
  if (B->status) (void)hipFree(B->status);
  for (auto& t : B->tiles)
    if (t) (void)hipFree(t);
  delete B;
}

grf_status grf_batch_rk4_stage(grf_batch* B, int stage, hipStream_t stream) {
  if (!B) return fail(GRF_EINVAL, "batch is null");
  if (stage < 1 || stage > 4) return fail(GRF_EINVAL, "stage must be 1..4 (got %d)", stage);
  return batch_stage(B, stage, stream);
}

grf_status grf_batch_step(grf_batch* B, hipStream_t stream) {
  if (!B) return fail(GRF_EINVAL, "batch is null");
  grf_status s;
  for (int stage = 1; stage <= 4; ++stage)
    if ((s = grf_batch_rk4_stage(B, stage, stream)) != GRF_OK) return s;
  return GRF_OK;
}

grf_status grf_batch_step_perbox(grf_batch* B, hipStream_t stream) {
  if (!B) return fail(GRF_EINVAL, "batch is null");
  const grf_point_params pp = make_pp(&B->params);
  const int sa = B->params.shift_advec != 0.0;
  for (int stage = 1; stage <= 4; ++stage) {
    const int mode = stage == 1 ? 1 : (stage == 4 ? 4 : 2);
    for (size_t b = 0; b < B->host.size(); ++b) {
      const BatchBoxDev& d = B->host[b];
      // the buffer roles of stage_roles: u -> ua -> ub -> ua -> u
      const double* in = stage == 1 ? d.u : (stage == 3 ? d.ub : d.ua);
      double* o = stage == 2 ? d.ub : (stage == 4 ? d.u : d.ua);
      const StageCoef sc{stage == 4 ? d.dt / 6.0 : (stage == 3 ? 1.0 * d.dt : 0.5 * d.dt)};
      prof_mark(0, stream);
      GRF_HIP_CHECK(launch_deriv(B->variant[b], d.bd, in, d.D, B->params.ko_sigma, sa, nullptr, stream));
      prof_mark(0, stream);
      prof_mark(1, stream);
      GRF_HIP_CHECK(launch_staged(mode, sa, d.bd, pp, in, d.D, d.u, o, d.acc, sc, B->status, stream));
      prof_mark(1, stream);
    }
  }
  return GRF_OK;
}

grf_status grf_batch_capture_step(grf_batch* B, hipStream_t stream, hipGraphExec_t* exec) {
  if (!B || !exec) return fail(GRF_EINVAL, "null argument");
  if (stream == 0) return fail(GRF_EINVAL, "capture needs a non-null stream");
  hipGraph_t graph;
  GRF_HIP_CHECK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  grf_status s = grf_batch_step(B, stream);
  hipError_t e = hipStreamEndCapture(stream, &graph);
  if (s != GRF_OK) return s;
  if (e != hipSuccess) return fail(GRF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(GRF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return GRF_OK;
}

grf_status grf_batch_autotune(grf_batch* B, hipStream_t stream) {
  if (!B) return fail(GRF_EINVAL, "batch is null");
  using Shape = std::tuple<int, int, int>;
  auto shape_of = [&](size_t b) { return std::make_tuple(B->boxes[b].nx, B->boxes[b].ny, B->boxes[b].nz); };
  bool all_cached = true;
  for (size_t b = 0; b < B->boxes.size(); ++b) all_cached = all_cached && g_tile_cache.count(shape_of(b));
  if (!all_cached) {
    hipEvent_t e0, e1;
    GRF_HIP_CHECK(hipEventCreate(&e0));
    GRF_HIP_CHECK(hipEventCreate(&e1));
    const int sa = B->params.shift_advec != 0.0;
    auto timed = [&](auto&& launch, float& best) -> grf_status {
      best = 1e30f;
      for (int rep_i = 0; rep_i < 4; ++rep_i) {
        GRF_HIP_CHECK(hipEventRecord(e0, stream));
        grf_status st = launch();
        if (st != GRF_OK) return st;
        GRF_HIP_CHECK(hipEventRecord(e1, stream));
        GRF_HIP_CHECK(hipEventSynchronize(e1));
        float t = 0.f;
        GRF_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
        if (rep_i > 0 && t < best) best = t;  // the first launch warms up
      }
      return GRF_OK;
    };
    // (1) per shape class: the variant fastest on one box of the class alone
    std::map<Shape, int> rep, mix;
    for (size_t b = 0; b < B->boxes.size(); ++b) rep.emplace(shape_of(b), (int)b);
    for (auto& kv : rep) {
      const BatchBoxDev& d = B->host[kv.second];
      int best = kBatchVariants[0];
      float best_t = 1e30f;
      for (int v : kBatchVariants) {
        float t;
        grf_status st = timed(
            [&]() -> grf_status {
              GRF_HIP_CHECK(launch_deriv(v, d.bd, d.u, d.D, B->params.ko_sigma, sa, nullptr, stream));
              return GRF_OK;
            },
            t);
        if (st != GRF_OK) return st;
        if (t < best_t) {  // strict: ties keep the earlier candidate
          best_t = t;
          best = v;
        }
      }
      mix[kv.first] = best;
    }
    // (2) whole assignments timed as the batched stencil stage runs them: the
    // per-class mix, then every variant for all boxes; boxes of one class run
    // concurrently with all others in one launch, so a variant that
    // loses on a box alone can win in the batch
    std::vector<std::vector<int>> cands;
    {
      std::vector<int> m(B->boxes.size());
      for (size_t b = 0; b < B->boxes.size(); ++b) m[b] = mix[shape_of(b)];
      cands.push_back(m);
    }
    for (int v : kBatchVariants) cands.push_back(std::vector<int>(B->boxes.size(), v));
    size_t best_c = 0;
    float best_t = 1e30f;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
      B->variant = cands[ci];
      grf_status st = batch_upload_tiles(B);
      if (st != GRF_OK) return st;
      float t;
      st = timed(
          [&]() -> grf_status {
            for (int v : kBatchVariants) {
              if (!B->ntiles[v]) continue;
              GRF_HIP_CHECK(launch_deriv_batch(v, B->grid_deriv[v], B->dev, B->tiles[v], B->ntiles[v], 1,
                                               B->params.ko_sigma, sa, stream));
            }
            return GRF_OK;
          },
          t);
      if (st != GRF_OK) return st;
      if (t < best_t) {
        best_t = t;
        best_c = ci;
      }
    }
    for (size_t b = 0; b < B->boxes.size(); ++b)
      if (!g_tile_cache.count(shape_of(b))) g_tile_cache[shape_of(b)] = cands[best_c][b];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  for (size_t b = 0; b < B->boxes.size(); ++b) B->variant[b] = g_tile_cache[shape_of(b)];
  return batch_upload_tiles(B);
}

grf_status grf_batch_state(const grf_batch* B, int box, double** current) {
  if (!B || !current || box < 0 || box >= (int)B->host.size()) return fail(GRF_EINVAL, "bad argument");
  *current = B->host[box].u;
  return GRF_OK;
}

grf_status grf_batch_tile_variant(const grf_batch* B, int box, int* variant) {
  if (!B || !variant || box < 0 || box >= (int)B->host.size()) return fail(GRF_EINVAL, "bad argument");
  *variant = B->variant[box];
  return GRF_OK;
}

grf_status grf_batch_set_tile_variant(grf_batch* B, int box, int variant) {
  if (!B || box < 0 || box >= (int)B->host.size()) return fail(GRF_EINVAL, "bad argument");
  bool ok = false;
  for (int v : kBatchVariants) ok = ok || v == variant;
  if (!ok) return fail(GRF_EINVAL, "variant %d cannot run batched", variant);
  B->variant[box] = variant;
  return batch_upload_tiles(B);
}

grf_status grf_graph_launch(hipGraphExec_t exec, hipStream_t stream) {
  if (!exec) return fail(GRF_EINVAL, "graph is null");
  GRF_HIP_CHECK(hipGraphLaunch(exec, stream));
  return GRF_OK;
}

grf_status grf_graph_destroy(hipGraphExec_t exec) {
  if (!exec) return fail(GRF_EINVAL, "graph is null");
  GRF_HIP_CHECK(hipGraphExecDestroy(exec));
  return GRF_OK;
}

grf_status grf_batch_status_fetch(const grf_batch* B, hipStream_t stream, uint32_t* bits) {
  if (!B) return fail(GRF_EINVAL, "batch is null");
  return grf_status_fetch(B->status, stream, bits);
}

// Start recording up to max_launches timed launches per kernel class.
grf_status grf_measure_peaks(void* scratch, size_t scratch_bytes, hipStream_t stream, double* fp64_tflops,
                             double* copy_gbps) {
  if (!scratch || !fp64_tflops || !copy_gbps) return fail(GRF_EINVAL, "null argument");
  const int64_t n = (int64_t)(scratch_bytes / 16);  // two halves of n doubles
  if (n < (1 << 20)) return fail(GRF_ENOMEM, "scratch below 16 MiB");
  int dev = 0, cus = 256;
  GRF_HIP_CHECK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  GRF_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  cus = prop.multiProcessorCount;
  double* x = (double*)scratch;
  double* y = x + n;
  hipEvent_t e0, e1;
  GRF_HIP_CHECK(hipEventCreate(&e0));
  GRF_HIP_CHECK(hipEventCreate(&e1));
  const int blocks = cus * 32;  // 32 workgroups of 256 threads per CU: many rounds of full occupancy
  const int iters = 4096;
  if (n < (int64_t)blocks * 256) return fail(GRF_ENOMEM, "scratch too small for the FMA probe");
  float best_f = 1e30f, best_c = 1e30f;
  for (int rep = 0; rep < 4; ++rep) {
    float t = 0.f;
    GRF_HIP_CHECK(hipEventRecord(e0, stream));
    GRF_HIP_CHECK(launch_fma_peak(blocks, iters, x, stream));
    GRF_HIP_CHECK(hipEventRecord(e1, stream));
    GRF_HIP_CHECK(hipEventSynchronize(e1));
    GRF_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
    if (rep > 0 && t < best_f) best_f = t;
    GRF_HIP_CHECK(hipEventRecord(e0, stream));
    GRF_HIP_CHECK(launch_copy_peak(cus * 64, n, x, y, stream));
    GRF_HIP_CHECK(hipEventRecord(e1, stream));
    GRF_HIP_CHECK(hipEventSynchronize(e1));
    GRF_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
    if (rep > 0 && t < best_c) best_c = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *fp64_tflops = (double)blocks * 256 * iters * kPeakChains * 2.0 / (best_f * 1e-3) / 1e12;
  *copy_gbps = 2.0 * (double)n * 8.0 / (best_c * 1e-3) / 1e9;
  return GRF_OK;
}

grf_status grf_prof_begin(int max_launches) {
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(GRF_EINVAL, "max_launches out of range");
  for (auto& c : g_prof.cls) {
    while ((int)c.ev.size() < 2 * max_launches) {
      hipEvent_t e;
      GRF_HIP_CHECK(hipEventCreate(&e));
      c.ev.push_back(e);
    }
    c.used = 0;
  }
  g_prof.cap = max_launches;
  g_prof.on = true;
  return GRF_OK;
}

// Stop recording; for each kernel class (0 stencil, 1 pointwise, 2 VJP, 3 the
// reverse pointwise kernel) return the summed kernel time in ms and the number
// of timed launches (waits for them).
grf_status grf_prof_end(double* ms, int* count) {
  g_prof.on = false;
  for (int k = 0; k < 4; ++k) {
    ProfClass& c = g_prof.cls[k];
    double tot = 0.0;
    for (int q = 0; q + 1 < c.used; q += 2) {
      GRF_HIP_CHECK(hipEventSynchronize(c.ev[q + 1]));
      float t = 0.f;
      GRF_HIP_CHECK(hipEventElapsedTime(&t, c.ev[q], c.ev[q + 1]));
      tot += t;
    }
    if (ms) ms[k] = tot;
    if (count) count[k] = c.used / 2;
    c.used = 0;
  }
  return GRF_OK;
}

// Select the stage path of the single-box calls: 0 the plain pointwise
// kernel, 2 the pointwise kernel with its inputs staged through LDS.
grf_status grf_set_stage_path(int path) {
  if (path != 0 && path != 2) return fail(GRF_EINVAL, "stage path must be 0 or 2");
  g_stage_path = path;
  return GRF_OK;
}

int grf_get_stage_path(void) { return g_stage_path; }
int grf_get_tile_variant(void) { return g_tile_variant; }

// Select the stencil variant (0..9) used by the single-box calls.
grf_status grf_set_tile_variant(int variant) {
  if (variant < -1 || variant >= kDerivVariants) return fail(GRF_EINVAL, "tile variant out of range");
  g_tile_variant = variant;
  return GRF_OK;
}

// Interior planes per z-slab of the split stage paths (0 = whole box).
grf_status grf_set_slab_planes(int planes) {
  if (planes < 0) return fail(GRF_EINVAL, "slab planes must be >= 0");
  g_slab_planes = planes;
  return GRF_OK;
}
int grf_get_slab_planes(void) { return g_slab_planes; }

}  // extern "C"
