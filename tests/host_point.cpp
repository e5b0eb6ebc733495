// Test-only host build of the generated pointwise algebra (forward and VJP, both
// shift-advection variants), so that the generated code can be checked against
// the CPU oracle without a GPU.
#include <cmath>
#include "gen_layout.h"

using std::fma;

template <bool SA>
static int rhs_point(const double* prm, const double* u, const double* D, double* rhs) {
  grf_point_params P;
  double* dst = reinterpret_cast<double*>(&P);
  for (unsigned q = 0; q < sizeof(P) / sizeof(double); ++q) dst[q] = prm[q];
  int bad = 0;
#define GRF_U(f) u[f]
#define GRF_D(c) D[c]
#define GRF_P(n) P.n
#define GRF_RHS(f, v) rhs[f] = (v)
#define GRF_PIVCHK(v) bad |= !(std::fabs(v) <= 1e12)
#define GRF_SHIFT_ADVEC SA
#include "gen_rhs.inc"
#undef GRF_SHIFT_ADVEC
#undef GRF_RHS
#undef GRF_PIVCHK
  return bad;
}

template <bool SA>
static void vjp_point(const double* prm, const double* u, const double* D, const double* w, double* ubar,
                      double* Dbar, double* thbar) {
  grf_point_params P;
  double* dst = reinterpret_cast<double*>(&P);
  for (unsigned q = 0; q < sizeof(P) / sizeof(double); ++q) dst[q] = prm[q];
#define GRF_W(f) w[f]
#define GRF_BAR_U(f, v) ubar[f] = (v)
#define GRF_BAR_D(c, v) Dbar[c] = (v)
#define GRF_BAR_TH(q, v) thbar[q] = (v)
#define GRF_SHIFT_ADVEC SA
#include "gen_vjp.inc"
#undef GRF_SHIFT_ADVEC
}

extern "C" int host_rhs_point(int sa, const double* prm, const double* u, const double* D, double* rhs) {
  return sa ? rhs_point<true>(prm, u, D, rhs) : rhs_point<false>(prm, u, D, rhs);
}

extern "C" void host_vjp_point(int sa, const double* prm, const double* u, const double* D, const double* w,
                               double* ubar, double* Dbar, double* thbar) {
  if (sa)
    vjp_point<true>(prm, u, D, w, ubar, Dbar, thbar);
  else
    vjp_point<false>(prm, u, D, w, ubar, Dbar, thbar);
}
