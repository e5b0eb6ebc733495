// CPU oracle for the 4dST + modified-CCZ4 right-hand side and its RK4 update.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// reference that the GPU library is checked against.  Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
// no code, header, table or constant generator with the HIP library.
//
// Everything is written as plain loops over tensor indices, templated on the
// scalar type so that the same source runs in double and in complex<double>
// (complex-step tangents).
//
// What is computed (the paper's Summary and Key features name the pieces; it
// prints no equations, so the equation set below is the covariant 4dST theory
// with backreaction written in 3+1 form):
//   * action (1/16pi) int sqrt(-g) [R + X + lambda(phi) L_GB + g2 X^2],
//     X = -1/2 (d phi)^2, lambda(phi) = lambda_lin phi + lambda_gb (1 -
//     exp(-beta phi^2)) / (4 beta) (the linear term: the shift-symmetric
//     coupling; beta = 0: lambda_gb phi^2 / 4), V = 0;
//   * CCZ4 with damping kappa1, kappa2, kappa3, the Z4 trace reversal done with
//     hat g^{mu nu} = g^{mu nu} - b n^mu n^nu (modified gauge function b);
//   * modified puncture gauge: 1+log lapse and B-form Gamma-driver, divided by
//     (1 + a) and with the -(a/(1+a)) alpha D^i alpha shift term (function a);
//   * the 4dST stress depends on C_ij = 4R_{i n j n} and on p = Lie_n Pi, which
//     enter the equations linearly: a 7x7 linear system per cell;
//   * 4th-order centred, mixed and lopsided-upwind finite differences, Kreiss-
//     Oliger dissipation sigma/(64 h) times the 6th difference, classic RK4;
//     sixth-order forms of the stencils on boxes with three ghost layers, and
//     on boxes with four ghost layers a sixth-order advection stencil and the
//     dissipation -sigma/(256 h) times the 8th difference.
// Readings taken where the paper is silent are marked "reading:" in the code.
//
// Conventions: 27 fields in the order
//   chi, h11 h12 h13 h22 h23 h33, K, A11 A12 A13 A22 A23 A33, Theta,
//   Gam1 Gam2 Gam3, lapse, shift1 shift2 shift3, B1 B2 B3, phi, Pi
// stored field-major [f][z][y][x] with 3 ghost cells on every side.

#include <cmath>
#include <complex>
#include <omp.h>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

using cplx = std::complex<double>;
inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }
inline bool finite_val(double x) { return std::isfinite(x); }
inline bool finite_val(const cplx& x) { return std::isfinite(x.real()) && std::isfinite(x.imag()); }
// extended precision (x87 80-bit: 64-bit significand), the reference that the
// double-precision results are measured against on ill-conditioned data
inline double re(long double x) { return (double)x; }
inline bool finite_val(long double x) { return std::isfinite(x); }

// ---------------------------------------------------------------- flop counting
// A scalar that records its own arithmetic on a tape, run through the same
// templated code to give the algorithmic flop count per cell used by roofline
// fractions.  One count each for +, -, *, / and for sqrt, cbrt, exp, pow;
// nothing for comparisons, negation, copies, abs and selects.  A value built
// from constants alone (literals, the double-typed parameters) is a constant:
// operations between constants are folded, as are additions of a constant 0
// and multiplications or divisions by a constant 0 or +-1, which are no
// arithmetic in any implementation.  Inputs (state values, couplings) are
// variables.  Only the operations that the requested outputs depend on are
// counted (values this code computes and never uses, such as second
// derivatives of fields that appear only with first derivatives, are not
// algorithmic work).
struct Flop {
  double v = 0.0;
  int32_t id = -1;  // -1 constant, -2 input variable, >= 0 tape node
  Flop() = default;
  Flop(double x) : v(x), id(-1) {}
  static Flop var(double x) {
    Flop f(x);
    f.id = -2;
    return f;
  }
};
struct FlopNode {
  int32_t a, b;
};
std::vector<FlopNode> g_tape;
inline Flop flop_node(double v, const Flop& a, const Flop& b) {
  Flop r(v);
  r.id = (int32_t)g_tape.size();
  g_tape.push_back(FlopNode{a.id, b.id});
  return r;
}
inline bool konst(const Flop& a) { return a.id == -1; }
inline bool unit(const Flop& a) { return konst(a) && (a.v == 1.0 || a.v == -1.0); }
inline Flop operator-(const Flop& a) {
  Flop r = a;
  r.v = -a.v;
  return r;
}
inline Flop operator+(const Flop& a, const Flop& b) {
  if (konst(a) && konst(b)) return Flop(a.v + b.v);
  if (konst(a) && a.v == 0.0) return b;
  if (konst(b) && b.v == 0.0) return a;
  return flop_node(a.v + b.v, a, b);
}
inline Flop operator-(const Flop& a, const Flop& b) {
  if (konst(a) && konst(b)) return Flop(a.v - b.v);
  if (konst(b) && b.v == 0.0) return a;
  if (konst(a) && a.v == 0.0) return -b;
  return flop_node(a.v - b.v, a, b);
}
inline Flop operator*(const Flop& a, const Flop& b) {
  if (konst(a) && konst(b)) return Flop(a.v * b.v);
  if ((konst(a) && a.v == 0.0) || (konst(b) && b.v == 0.0)) return Flop(0.0);
  if (unit(a)) return a.v > 0 ? b : -b;
  if (unit(b)) return b.v > 0 ? a : -a;
  return flop_node(a.v * b.v, a, b);
}
inline Flop operator/(const Flop& a, const Flop& b) {
  if (konst(a) && konst(b)) return Flop(a.v / b.v);
  if (konst(a) && a.v == 0.0) return Flop(0.0);
  if (unit(b)) return b.v > 0 ? a : -a;
  return flop_node(a.v / b.v, a, b);
}
inline Flop& operator+=(Flop& a, const Flop& b) { return a = a + b; }
inline Flop& operator-=(Flop& a, const Flop& b) { return a = a - b; }
inline Flop& operator*=(Flop& a, const Flop& b) { return a = a * b; }
inline Flop& operator/=(Flop& a, const Flop& b) { return a = a / b; }
#define GRF_FLOP_MIXED(op)                                                        \
  inline Flop operator op(const Flop& a, double b) { return a op Flop(b); }      \
  inline Flop operator op(double a, const Flop& b) { return Flop(a) op b; }      \
  inline Flop operator op(const Flop& a, int b) { return a op Flop(double(b)); } \
  inline Flop operator op(int a, const Flop& b) { return Flop(double(a)) op b; }
GRF_FLOP_MIXED(+)
GRF_FLOP_MIXED(-)
GRF_FLOP_MIXED(*)
GRF_FLOP_MIXED(/)
#undef GRF_FLOP_MIXED
inline Flop flop_fn(double v, const Flop& a) { return konst(a) ? Flop(v) : flop_node(v, a, Flop()); }
inline Flop sqrt(const Flop& a) { return flop_fn(std::sqrt(a.v), a); }
inline Flop cbrt(const Flop& a) { return flop_fn(std::cbrt(a.v), a); }
inline Flop exp(const Flop& a) { return flop_fn(std::exp(a.v), a); }
inline Flop pow(const Flop& a, double e) { return flop_fn(std::pow(a.v, e), a); }
inline Flop abs(const Flop& a) {
  Flop r = a;
  r.v = std::fabs(a.v);
  return r;
}
inline double re(const Flop& x) { return x.v; }
inline bool finite_val(const Flop& x) { return std::isfinite(x.v); }
// Number of tape operations that the given outputs depend on.
int64_t flop_count_live(const std::vector<int32_t>& outputs) {
  std::vector<char> live(g_tape.size(), 0);
  for (int32_t o : outputs)
    if (o >= 0) live[o] = 1;
  int64_t n = 0;
  for (int64_t q = (int64_t)g_tape.size() - 1; q >= 0; --q) {
    if (!live[q]) continue;
    ++n;
    if (g_tape[q].a >= 0) live[g_tape[q].a] = 1;
    if (g_tape[q].b >= 0) live[g_tape[q].b] = 1;
  }
  return n;
}

enum {
  CHI = 0, H11 = 1, KTR = 7, A11 = 8, THETA = 14, GH1 = 15, LAPSE = 18, SHIFT1 = 19,
  BB1 = 22, PHI = 25, PI_ = 26, NF = 27
};
// symmetric 3x3 index -> packed position (xx, xy, xz, yy, yz, zz)
const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

// Levi-Civita permutation symbol
int eps3(int a, int b, int c) {
  if (a == b || b == c || a == c) return 0;
  // even permutations of (0,1,2)
  if ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) || (a == 2 && b == 0 && c == 1)) return 1;
  return -1;
}
// generalised Kronecker delta  delta^{abc}_{def} = eps^{abc} eps_{def}
int gdelta(int a, int b, int c, int d, int e, int f) { return eps3(a, b, c) * eps3(d, e, f); }

// Flag bits reported per cell.
enum { FLAG_NONFINITE = 1, FLAG_HYPERBOLIC = 2, FLAG_NONPOSITIVE = 4 };

template <class T>
struct Params {
  T lambda_gb;           // lambda(phi) = lambda_gb * phi^2 / 4
  T g2;                  // constant coefficient of X^2
  double a, b;           // modified-gauge functions a(x), b(x) (constants)
  double kappa1, kappa2, kappa3;
  double lapse_coeff, lapse_power, lapse_advec;
  double shift_gamma_coeff, shift_advec, eta;
  double ko_sigma;
  double decoupled;      // 1: decoupling limit, the scalar does not source the metric
  int fd_order;          // 4 or 6: order of the centred finite differences
  double lambda_lin;     // linear (shift-symmetric) part of lambda(phi)
  double beta;           // exponential form of the even part of lambda(phi) (0: quadratic)
};

template <class T>
T det3(const T m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

template <class T>
void inv3(const T m[3][3], T out[3][3]) {
  const T d = det3(m);
  out[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / d;
  out[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / d;
  out[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / d;
  out[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / d;
  out[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / d;
  out[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / d;
  out[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / d;
  out[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / d;
  out[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / d;
}

// Dense linear solve by Gaussian elimination with partial pivoting (any stable
// solver will do for the oracle).  Returns the smallest |pivot| / (max-norm of
// its row) seen, so the caller can flag near-singular systems.
template <class T>
double gepp_solve(int n, T* A /* n*n row-major, destroyed */, T* b /* n, destroyed */, T* x, T* det = nullptr) {
  double worst = 1e300;
  int swaps = 0;
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(re(A[k * n + k]));
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(re(A[i * n + k]));
      if (v > best) { best = v; p = i; }
    }
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(b[k], b[p]);
      ++swaps;
    }
    double rownorm = 0.0;
    for (int j = k; j < n; ++j) rownorm = std::max(rownorm, std::abs(re(A[k * n + j])));
    double ratio = rownorm > 0 ? std::abs(re(A[k * n + k])) / rownorm : 0.0;
    worst = std::min(worst, ratio);
    for (int i = k + 1; i < n; ++i) {
      T f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
    x[i] = s / A[i * n + i];
  }
  if (det) {  // determinant: product of the pivots, sign of the row exchanges
    T d = (swaps % 2) ? T(-1.0) : T(1.0);
    for (int k = 0; k < n; ++k) d *= A[k * n + k];
    *det = d;
  }
  return worst;
}

// Everything the pointwise right-hand side needs at one cell.
template <class T>
struct PointIn {
  T u[NF];
  T d1[NF][3];   // centred first derivatives d_k u_f
  T d2[NF][6];   // centred second derivatives d_k d_l u_f, packed (xx,xy,xz,yy,yz,zz)
  T adv[NF][3];  // upwinded first derivatives along each axis (side chosen by sign of shift)
};

template <class T>
struct PointOut {
  T rhs[NF];
  T ham;          // Hamiltonian constraint  R + 2/3 K^2 - A_ij A^ij - 2 (8 pi rho)
  T mom[3];       // momentum constraint  M_i - 8 pi S_i
  T rho[3];       // energy density n^a n^b T_ab of the canonical (X), X^2 and Gauss-Bonnet terms
  T lgb;          // Gauss-Bonnet invariant of the spacetime (with the solved C_ij)
  T weak[2];      // weak-coupling indicators |lambda'(phi)| sqrt|L_GB| and |2 g2 X|
  T detA;         // determinant of the per-cell system (zero where the time derivatives cannot be solved for)
  T C[6];         // solved C_ij = 4R_{i n j n}
  T p;            // solved Lie_n Pi
  T sysA[49];     // the assembled 7x7 system (row-major), for solver checks
  T sysb[7];
  double pivot_ratio;
  int flags;
};

// Pointwise 4dST + modified CCZ4 right-hand side (without Kreiss-Oliger).
template <class T>
void rhs_point(const Params<T>& P, const PointIn<T>& in, PointOut<T>& out) {
  const T* u = in.u;
  const T chi = u[CHI];
  const T K = u[KTR];
  const T Th = u[THETA];
  const T alpha = u[LAPSE];
  const T phi = u[PHI];
  const T Pi = u[PI_];
  T h[3][3], A[3][3];
  T Gh[3], beta[3], Bv[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      h[i][j] = u[H11 + SYM[i][j]];
      A[i][j] = u[A11 + SYM[i][j]];
    }
  for (int i = 0; i < 3; ++i) {
    Gh[i] = u[GH1 + i];
    beta[i] = u[SHIFT1 + i];
    Bv[i] = u[BB1 + i];
  }

  // ---- first and second derivatives, unpacked
  T dchi[3], dK[3], dTh[3], dalpha[3], dphi[3], dPi[3];
  T dh[3][3][3];     // dh[k][i][j] = d_k h_ij
  T dA[3][3][3];     // dA[k][i][j] = d_k A_ij
  T dGh[3][3];       // dGh[i][k] = d_k Gh^i
  T dbeta[3][3];     // dbeta[i][k] = d_k beta^i
  T ddchi[3][3], ddalpha[3][3], ddphi[3][3];
  T ddh[3][3][3][3];  // ddh[k][l][i][j] = d_k d_l h_ij
  T ddbeta[3][3][3];  // ddbeta[i][k][l] = d_k d_l beta^i
  for (int k = 0; k < 3; ++k) {
    dchi[k] = in.d1[CHI][k];
    dK[k] = in.d1[KTR][k];
    dTh[k] = in.d1[THETA][k];
    dalpha[k] = in.d1[LAPSE][k];
    dphi[k] = in.d1[PHI][k];
    dPi[k] = in.d1[PI_][k];
    for (int i = 0; i < 3; ++i) {
      dGh[i][k] = in.d1[GH1 + i][k];
      dbeta[i][k] = in.d1[SHIFT1 + i][k];
      for (int j = 0; j < 3; ++j) {
        dh[k][i][j] = in.d1[H11 + SYM[i][j]][k];
        dA[k][i][j] = in.d1[A11 + SYM[i][j]][k];
      }
    }
    for (int l = 0; l < 3; ++l) {
      ddchi[k][l] = in.d2[CHI][SYM[k][l]];
      ddalpha[k][l] = in.d2[LAPSE][SYM[k][l]];
      ddphi[k][l] = in.d2[PHI][SYM[k][l]];
      for (int i = 0; i < 3; ++i) {
        ddbeta[i][k][l] = in.d2[SHIFT1 + i][SYM[k][l]];
        for (int j = 0; j < 3; ++j) ddh[k][l][i][j] = in.d2[H11 + SYM[i][j]][SYM[k][l]];
      }
    }
  }

  int flags = 0;
  if (re(chi) <= 0.0 || re(alpha) <= 0.0) flags |= FLAG_NONPOSITIVE;

  // ---- conformal metric inverse and Christoffel symbols
  T hu[3][3];
  inv3(h, hu);
  T chr1[3][3][3];  // Gamma~_{kij} = 1/2 (d_i h_kj + d_j h_ki - d_k h_ij)
  T chr[3][3][3];   // Gamma~^k_{ij}
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) chr1[k][i][j] = 0.5 * (dh[i][k][j] + dh[j][k][i] - dh[k][i][j]);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T s = 0.0;
        for (int l = 0; l < 3; ++l) s += hu[k][l] * chr1[l][i][j];
        chr[k][i][j] = s;
      }
  T Gt[3];  // Gamma~^k = h^ij Gamma~^k_ij
  for (int k = 0; k < 3; ++k) {
    T s = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) s += hu[i][j] * chr[k][i][j];
    Gt[k] = s;
  }
  // Z vector: Z~^k = 1/2 (Gh^k - Gamma~^k), physical covector Z_i = h_ik Z~^k
  T Zt[3], Zl[3];
  for (int k = 0; k < 3; ++k) Zt[k] = 0.5 * (Gh[k] - Gt[k]);
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int k = 0; k < 3; ++k) s += h[i][k] * Zt[k];
    Zl[i] = s;
  }
  // physical Christoffel symbols of gamma_ij = h_ij / chi
  T chrp[3][3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T hud = 0.0;  // h^kl d_l chi
        for (int l = 0; l < 3; ++l) hud += hu[k][l] * dchi[l];
        T corr = (k == i ? dchi[j] : T(0.0)) + (k == j ? dchi[i] : T(0.0)) - h[i][j] * hud;
        chrp[k][i][j] = chr[k][i][j] - corr / (2.0 * chi);
      }
  // physical metric and inverse
  T gam[3][3], gu[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gam[i][j] = h[i][j] / chi;
      gu[i][j] = chi * hu[i][j];
    }

  // ---- D_i D_j alpha and its trace
  T DDa[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = ddalpha[i][j];
      for (int k = 0; k < 3; ++k) s -= chrp[k][i][j] * dalpha[k];
      DDa[i][j] = s;
    }
  T D2a = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D2a += gu[i][j] * DDa[i][j];

  // ---- derivatives of the conformal connection, for the pure Ricci tensor
  T dhu[3][3][3];  // dhu[j][l][m] = d_j h^lm = - h^la h^mb d_j h_ab
  for (int j = 0; j < 3; ++j)
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m) {
        T s = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s -= hu[l][a] * hu[m][b] * dh[j][a][b];
        dhu[j][l][m] = s;
      }
  T dchr[3][3][3][3];  // dchr[j][k][l][m] = d_j Gamma~^k_lm
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) {
          T s = 0.0;
          for (int n = 0; n < 3; ++n) {
            s += dhu[j][k][n] * chr1[n][l][m];
            s += hu[k][n] * 0.5 * (ddh[j][l][n][m] + ddh[j][m][n][l] - ddh[j][n][l][m]);
          }
          dchr[j][k][l][m] = s;
        }
  T dGt[3][3];  // dGt[k][j] = d_j Gamma~^k
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) s += dhu[j][l][m] * chr[k][l][m] + hu[l][m] * dchr[j][k][l][m];
      dGt[k][j] = s;
    }

  // conformal Ricci tensor written with a given contracted connection G^k and its derivative
  auto ricci_tilde = [&](const T G[3], const T dG[3][3], T out_r[3][3]) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T s = 0.0;
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < 3; ++m) s += -0.5 * hu[l][m] * ddh[l][m][i][j];
        for (int k = 0; k < 3; ++k) s += 0.5 * (h[k][i] * dG[k][j] + h[k][j] * dG[k][i]);
        for (int k = 0; k < 3; ++k) s += 0.5 * G[k] * (chr1[i][j][k] + chr1[j][i][k]);
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < 3; ++m)
            for (int k = 0; k < 3; ++k)
              s += hu[l][m] * (chr[k][l][i] * chr1[j][k][m] + chr[k][l][j] * chr1[i][k][m] +
                               chr[k][i][m] * chr1[k][l][j]);
        out_r[i][j] = s;
      }
  };
  T RtGh[3][3], RtGt[3][3];
  ricci_tilde(Gh, dGh, RtGh);
  ricci_tilde(Gt, dGt, RtGt);

  // chi part of the Ricci tensor
  T DDchi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = ddchi[i][j];
      for (int k = 0; k < 3; ++k) s -= chr[k][i][j] * dchi[k];
      DDchi[i][j] = s;
    }
  T trDDchi = 0.0, dchi2 = 0.0;
  for (int l = 0; l < 3; ++l)
    for (int m = 0; m < 3; ++m) {
      trDDchi += hu[l][m] * DDchi[l][m];
      dchi2 += hu[l][m] * dchi[l] * dchi[m];
    }
  T Rchi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Rchi[i][j] = (DDchi[i][j] + h[i][j] * trDDchi) / (2.0 * chi) -
                   (dchi[i] * dchi[j] + 3.0 * h[i][j] * dchi2) / (4.0 * chi * chi);
  T Ztdchi = 0.0;
  for (int l = 0; l < 3; ++l) Ztdchi += Zt[l] * dchi[l];
  T Rz[3][3], Rp[3][3];  // R_ij + 2 D_(i Z_j)   and pure R_ij
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Rz[i][j] = RtGh[i][j] + Rchi[i][j] + (Zl[i] * dchi[j] + Zl[j] * dchi[i] - h[i][j] * Ztdchi) / chi;
      Rp[i][j] = RtGt[i][j] + Rchi[i][j];
    }
  T Rzs = 0.0, Rs = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Rzs += gu[i][j] * Rz[i][j];
      Rs += gu[i][j] * Rp[i][j];
    }

  // ---- extrinsic curvature pieces
  T Au[3][3];   // A~^ij
  T Aud[3][3];  // A~^i_j = h^ik A_kj
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0, s2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        s2 += hu[i][k] * A[k][j];
        for (int l = 0; l < 3; ++l) s += hu[i][k] * hu[j][l] * A[k][l];
      }
      Au[i][j] = s;
      Aud[i][j] = s2;
    }
  T A2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A2 += A[i][j] * Au[i][j];
  // momentum constraint  M_i = D_j K^j_i - D_i K
  T Mi[3];
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        T t = dA[k][j][i];
        for (int l = 0; l < 3; ++l) t -= chr[l][k][j] * A[l][i] + chr[l][k][i] * A[j][l];
        s += hu[j][k] * t;
      }
    for (int k = 0; k < 3; ++k) s -= 1.5 * Aud[k][i] * dchi[k] / chi;
    s -= (2.0 / 3.0) * dK[i];
    Mi[i] = s;
  }
  // physical K_ij, K^i_j, derivatives
  T Kl[3][3], Kud[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Kl[i][j] = (A[i][j] + h[i][j] * K / 3.0) / chi;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int k = 0; k < 3; ++k) s += gu[i][k] * Kl[k][j];
      Kud[i][j] = s;
    }
  T dKl[3][3][3];  // d_k K_ij
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        dKl[k][i][j] = (dA[k][i][j] + dh[k][i][j] * K / 3.0 + h[i][j] * dK[k] / 3.0) / chi -
                       (A[i][j] + h[i][j] * K / 3.0) * dchi[k] / (chi * chi);
  T DK[3][3][3];  // DK[k][i][j] = D_k K_ij
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T s = dKl[k][i][j];
        for (int l = 0; l < 3; ++l) s -= chrp[l][k][i] * Kl[l][j] + chrp[l][k][j] * Kl[i][l];
        DK[k][i][j] = s;
      }
  T Bt[3][3][3];  // B_ijk = D_j K_ik - D_k K_ij
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) Bt[i][j][k] = DK[j][i][k] - DK[k][i][j];

  // spatial projection of the Riemann tensor (Gauss): A_ij = R_ij + K K_ij - K_ik K^k_j
  T A4[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = Rp[i][j] + K * Kl[i][j];
      for (int k = 0; k < 3; ++k) s -= Kl[i][k] * Kud[k][j];
      A4[i][j] = s;
    }
  const T A4tr = Rs + (2.0 / 3.0) * K * K - A2;
  T Gc[3][3];   // curly G_ij
  T Gcu[3][3];  // G^ij
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Gc[i][j] = A4[i][j] - 0.5 * gam[i][j] * A4tr;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s += gu[i][a] * gu[j][b] * Gc[a][b];
      Gcu[i][j] = s;
    }
  T Gctr = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Gctr += gu[i][j] * Gc[i][j];

  // ---- scalar field pieces
  T dphiu[3];
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int j = 0; j < 3; ++j) s += gu[i][j] * dphi[j];
    dphiu[i] = s;
  }
  T dphi2 = 0.0;
  for (int i = 0; i < 3; ++i) dphi2 += dphi[i] * dphiu[i];
  const T X = 0.5 * (Pi * Pi - dphi2);
  const T g2 = P.g2;
  const T FX = 1.0 + 2.0 * g2 * X;
  const T F = X + g2 * X * X;               // V = 0
  // lambda(phi) = lambda_lin phi + lambda_gb (1 - exp(-beta phi^2)) / (4 beta)
  // (beta -> 0: lambda_gb phi^2 / 4); only its first two derivatives enter
  using std::exp;
  const T ex = exp(-P.beta * phi * phi);
  const T dlam = P.lambda_lin + 0.5 * P.lambda_gb * phi * ex;               // lambda'(phi)
  const T ddlam = 0.5 * P.lambda_gb * (1.0 - 2.0 * P.beta * phi * phi) * ex;  // lambda''(phi)
  T DDphi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = ddphi[i][j];
      for (int k = 0; k < 3; ++k) s -= chrp[k][i][j] * dphi[k];
      DDphi[i][j] = s;
    }
  T al[3], au[3];  // a_i = d_i ln alpha, a^i
  for (int i = 0; i < 3; ++i) al[i] = dalpha[i] / alpha;
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int j = 0; j < 3; ++j) s += gu[i][j] * al[j];
    au[i] = s;
  }
  T adphi = 0.0;
  for (int k = 0; k < 3; ++k) adphi += au[k] * dphi[k];
  T W[3][3], Vl[3], Vu[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) W[i][j] = dlam * (DDphi[i][j] + Kl[i][j] * Pi) + ddlam * dphi[i] * dphi[j];
  for (int i = 0; i < 3; ++i) {
    T s = dPi[i];
    for (int j = 0; j < 3; ++j) s += Kud[j][i] * dphi[j];  // K_i^j d_j phi
    Vl[i] = dlam * s + ddlam * Pi * dphi[i];
  }
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int j = 0; j < 3; ++j) s += gu[i][j] * Vl[j];
    Vu[i] = s;
  }
  const T Wnn0 = -dlam * adphi + ddlam * Pi * Pi;  // W_nn = lambda' p + Wnn0

  // raised pieces of B_ijk
  T Bsup[3][3][3];  // B^s_ab = g^sm B_mab
  T Bdup[3][3][3];  // B_b^{rs} = B_bmn g^mr g^ns
  for (int s = 0; s < 3; ++s)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        T t = 0.0;
        for (int m = 0; m < 3; ++m) t += gu[s][m] * Bt[m][a][b];
        Bsup[s][a][b] = t;
      }
  for (int b = 0; b < 3; ++b)
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        T t = 0.0;
        for (int m = 0; m < 3; ++m)
          for (int n = 0; n < 3; ++n) t += Bt[b][m][n] * gu[m][r] * gu[n][s];
        Bdup[b][r][s] = t;
      }
  T B2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        T t = 0.0;
        for (int a = 0; a < 3; ++a) t += gu[i][a] * Bdup[a][j][k];
        B2 += Bt[i][j][k] * t;
      }
  T M2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M2 += Mi[i] * gu[i][j] * Mi[j];

  // the part of H_ij that does not depend on (C, p): the B.V terms
  T HBV[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int e = 0; e < 3; ++e) {
        T t = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            for (int d = 0; d < 3; ++d)
              for (int q = 0; q < 3; ++q) {
                int g1 = gdelta(e, a, b, j, d, q);
                if (g1) t += double(g1) * Bsup[q][a][b] * Vu[d];
              }
        for (int c = 0; c < 3; ++c)
          for (int b = 0; b < 3; ++b)
            for (int r = 0; r < 3; ++r)
              for (int q = 0; q < 3; ++q) {
                int g1 = gdelta(e, c, b, j, r, q);
                if (g1) t += double(g1) * Bdup[b][r][q] * Vl[c];
              }
        s += 2.0 * gam[i][e] * t;
      }
      HBV[i][j] = s;
    }

  // bilinear bracket of H_ij in C and W:
  //  gamma_ij (trC trW - tr(CW)) - trC W_ij - trW C_ij + (CW)_ij + (WC)_ij
  T trW = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trW += gu[i][j] * W[i][j];
  auto bracket = [&](const T C[3][3], T out_b[3][3]) {
    T trC = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) trC += gu[i][j] * C[i][j];
    T CW[3][3], WC[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) {
            s1 += C[i][k] * gu[k][l] * W[l][j];
            s2 += W[i][k] * gu[k][l] * C[l][j];
          }
        CW[i][j] = s1;
        WC[i][j] = s2;
      }
    T trCW = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) trCW += CW[i][j] * gu[j][i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        out_b[i][j] = gam[i][j] * (trC * trW - trCW) - trC * W[i][j] - trW * C[i][j] + CW[i][j] + WC[i][j];
  };
  // full H_ij(C, p)
  auto Hfull = [&](const T C[3][3], const T p, T out_h[3][3]) {
    T br[3][3];
    bracket(C, br);
    const T Wnn = dlam * p + Wnn0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) out_h[i][j] = 4.0 * Gc[i][j] * Wnn - 4.0 * br[i][j] + HBV[i][j];
  };
  auto trace_rev = [&](const T M[3][3], T out_m[3][3]) {  // M_ij - 1/2 gamma_ij gamma^kl M_kl
    T tr = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) tr += gu[k][l] * M[k][l];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) out_m[i][j] = M[i][j] - 0.5 * gam[i][j] * tr;
  };

  // H^0_i and H^0_0, energy density, momentum density
  T H0i[3];
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int c = 0; c < 3; ++c) {
      T Gic = 0.0;  // G_i^c
      for (int k = 0; k < 3; ++k) Gic += Gc[i][k] * gu[k][c];
      s += -4.0 * Gic * Vl[c];
    }
    for (int c = 0; c < 3; ++c)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 3; ++q) {
              int g1 = gdelta(c, a, b, i, d, q);
              if (!g1) continue;
              T Wdc = 0.0;  // W^d_c
              for (int k = 0; k < 3; ++k) Wdc += gu[d][k] * W[k][c];
              s += -2.0 * double(g1) * Bsup[q][a][b] * Wdc;
            }
    H0i[i] = s;
  }
  T GW = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GW += Gcu[i][j] * W[i][j];
  const T H00 = -4.0 * GW;
  const T rho8 = 0.5 * FX * Pi * Pi - 0.5 * F + H00;  // 8 pi rho
  T S8i[3];
  for (int i = 0; i < 3; ++i) S8i[i] = -0.5 * FX * Pi * dphi[i] - H0i[i];
  T Sig[3][3];  // scalar stress Sigma_ij
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Sig[i][j] = 0.5 * FX * dphi[i] * dphi[j] + 0.5 * gam[i][j] * F;
  T Sigtr = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Sigtr += gu[i][j] * Sig[i][j];
  // Decoupling limit (Key features, "Modified gravity theories": 4dST without
  // backreaction): the scalar moves on the metric but does not source it, so
  // the metric equations see no energy, momentum, stress or Gauss-Bonnet
  // tensor and the metric rows of the system below reduce to C_ij = Q_ij.
  const bool dec = P.decoupled != 0.0;
  const T rho8m = dec ? T(0.0) : rho8;
  T S8im[3], Sigm[3][3];
  for (int i = 0; i < 3; ++i) {
    S8im[i] = dec ? T(0.0) : S8i[i];
    for (int j = 0; j < 3; ++j) Sigm[i][j] = dec ? T(0.0) : Sig[i][j];
  }
  const T Sigtrm = dec ? T(0.0) : Sigtr;

  // ---- the per-cell linear system for (C_ij, p)
  const double bb = P.b, aa = P.a;
  const double cfac = 1.0 / (1.0 + bb);
  const double k1 = P.kappa1, k2 = P.kappa2, k3 = P.kappa3;
  // reading: the b-terms and the 4dST curvature use the Ricci tensor without the Z terms
  const T Hg = Rs + (2.0 / 3.0) * K * K - A2;  // R + K^2 - K_ij K^ij
  T Q[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = Rz[i][j] + (K - 2.0 * Th) * Kl[i][j];
      for (int k = 0; k < 3; ++k) s -= Kl[i][k] * Kud[k][j];
      s += -Sigm[i][j] + 0.5 * gam[i][j] * Sigtrm;
      s -= gam[i][j] * ((bb / (4.0 * (1.0 + bb))) * Hg + 0.5 * cfac * rho8m +
                        0.5 * cfac * k1 * (2.0 + k2) * Th + 0.5 * k1 * k2 * Th);
      Q[i][j] = s;
    }
  // scalar equation, everything except lambda' 8 G^ij C_ij and the p term
  T KDD = 0.0, PiV = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) KDD += dphiu[i] * dphiu[j] * (DDphi[i][j] + Kl[i][j] * Pi);
  for (int i = 0; i < 3; ++i) {
    T s = dPi[i];
    for (int j = 0; j < 3; ++j) s += Kud[j][i] * dphi[j];
    PiV += dphiu[i] * s;
  }
  T D2phi = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D2phi += gu[i][j] * DDphi[i][j];
  const T DPi = 1.0 + 3.0 * g2 * Pi * Pi - g2 * dphi2;
  const T srest = FX * (D2phi + K * Pi + adphi) - 2.0 * g2 * (KDD - 2.0 * Pi * PiV - Pi * Pi * adphi);
  const T s_rhs = srest + dlam * (-4.0 * B2 + 8.0 * M2);

  T Amat[49], bvec[7];
  {
    // columns for the six C components (symmetric unit tensors)
    const int ci[6] = {0, 0, 0, 1, 1, 2}, cj[6] = {0, 1, 2, 1, 2, 2};
    for (int col = 0; col < 6; ++col) {
      T E[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) E[i][j] = 0.0;
      E[ci[col]][cj[col]] = 1.0;
      E[cj[col]][ci[col]] = 1.0;
      T br[3][3], Hl[3][3], Hr[3][3];
      bracket(E, br);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Hl[i][j] = -4.0 * br[i][j];
      trace_rev(Hl, Hr);
      for (int row = 0; row < 6; ++row) {
        const int i = ci[row], j = cj[row];
        Amat[row * 7 + col] = dec ? E[i][j] : E[i][j] - Hr[i][j];
      }
      T gE = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gE += Gcu[i][j] * E[i][j];
      Amat[6 * 7 + col] = -8.0 * dlam * gE;
    }
    // column for p
    {
      T Hl[3][3], Hr[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Hl[i][j] = 4.0 * Gc[i][j] * dlam;
      trace_rev(Hl, Hr);
      for (int row = 0; row < 6; ++row) Amat[row * 7 + 6] = dec ? T(0.0) : -Hr[ci[row]][cj[row]];
      Amat[6 * 7 + 6] = DPi;
    }
    // right-hand side: Q_ij + trace-reversed constant part of H
    T H0[3][3], H0r[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H0[i][j] = 4.0 * Gc[i][j] * Wnn0 + HBV[i][j];
    trace_rev(H0, H0r);
    for (int row = 0; row < 6; ++row) bvec[row] = dec ? Q[ci[row]][cj[row]] : Q[ci[row]][cj[row]] + H0r[ci[row]][cj[row]];
    bvec[6] = s_rhs;
  }
  for (int q = 0; q < 49; ++q) out.sysA[q] = Amat[q];
  for (int q = 0; q < 7; ++q) out.sysb[q] = bvec[q];
  T Awork[49], bwork[7], xs[7];
  for (int q = 0; q < 49; ++q) Awork[q] = Amat[q];
  for (int q = 0; q < 7; ++q) bwork[q] = bvec[q];
  T detA;
  const double pr = gepp_solve(7, Awork, bwork, xs, &detA);
  out.detA = detA;
  out.pivot_ratio = pr;
  if (!(pr >= 1e-12)) flags |= FLAG_HYPERBOLIC;
  T Cs[3][3];
  {
    const int ci[6] = {0, 0, 0, 1, 1, 2}, cj[6] = {0, 1, 2, 1, 2, 2};
    for (int q = 0; q < 6; ++q) {
      Cs[ci[q]][cj[q]] = xs[q];
      Cs[cj[q]][ci[q]] = xs[q];
      out.C[q] = xs[q];
    }
  }
  const T ps = xs[6];
  out.p = ps;
  T Hs[3][3], S8[3][3];
  Hfull(Cs, ps, Hs);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S8[i][j] = dec ? T(0.0) : Sig[i][j] - Hs[i][j];
  T S8tr = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S8tr += gu[i][j] * S8[i][j];

  // ---- right-hand sides
  T adv[NF];
  for (int f = 0; f < NF; ++f) {
    T s = 0.0;
    for (int k = 0; k < 3; ++k) s += beta[k] * in.adv[f][k];
    adv[f] = s;
  }
  T divb = 0.0;
  for (int k = 0; k < 3; ++k) divb += dbeta[k][k];
  const double fb = bb / (1.0 + bb);
  const T Hcal = Hg - 2.0 * rho8m - 2.0 * k1 * (2.0 + k2) * Th;

  T* r = out.rhs;
  r[CHI] = adv[CHI] + (2.0 / 3.0) * chi * (alpha * K - divb);
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      T s = adv[H11 + SYM[i][j]];
      for (int k = 0; k < 3; ++k) s += h[k][i] * dbeta[k][j] + h[k][j] * dbeta[k][i];
      s += -(2.0 / 3.0) * h[i][j] * divb - 2.0 * alpha * A[i][j];
      r[H11 + SYM[i][j]] = s;
    }
  r[KTR] = adv[KTR] - D2a + alpha * (Rzs + K * (K - 2.0 * Th)) - 3.0 * alpha * k1 * (1.0 + k2) * Th +
           0.5 * alpha * (S8tr - 3.0 * rho8m) - 0.75 * alpha * fb * Hcal;
  {
    T Xm[3][3];  // -D_i D_j alpha + alpha (Rz_ij - 8 pi S_ij)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Xm[i][j] = -DDa[i][j] + alpha * (Rz[i][j] - S8[i][j]);
    T trX = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) trX += hu[k][l] * Xm[k][l];
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) {
        T s = adv[A11 + SYM[i][j]];
        for (int k = 0; k < 3; ++k) s += A[k][i] * dbeta[k][j] + A[k][j] * dbeta[k][i];
        s += -(2.0 / 3.0) * A[i][j] * divb;
        s += chi * (Xm[i][j] - h[i][j] * trX / 3.0);
        T AA = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) AA += A[i][k] * hu[k][l] * A[l][j];
        s += alpha * (A[i][j] * (K - 2.0 * Th) - 2.0 * AA);
        r[A11 + SYM[i][j]] = s;
      }
  }
  {
    T Zda = 0.0;
    for (int k = 0; k < 3; ++k) Zda += Zt[k] * dalpha[k];
    r[THETA] = adv[THETA] + 0.5 * alpha * (Rzs - A2 + (2.0 / 3.0) * K * K - 2.0 * Th * K) - chi * Zda -
               alpha * k1 * (2.0 + k2) * Th - alpha * rho8m - 0.5 * alpha * fb * Hcal;
  }
  T rGam[3];
  for (int i = 0; i < 3; ++i) {
    T s = adv[GH1 + i];
    for (int k = 0; k < 3; ++k) s -= Gt[k] * dbeta[i][k];
    s += (2.0 / 3.0) * Gt[i] * divb;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) s += hu[j][k] * ddbeta[i][j][k] + hu[i][j] * ddbeta[k][j][k] / 3.0;
    {
      T zb = 0.0;
      for (int k = 0; k < 3; ++k) zb += Zt[k] * dbeta[i][k];
      s += 2.0 * k3 * ((2.0 / 3.0) * Zt[i] * divb - zb);
    }
    {
      T t = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) t += chr[i][j][k] * Au[j][k];
      for (int j = 0; j < 3; ++j) t -= 1.5 * Au[i][j] * dchi[j] / chi + (2.0 / 3.0) * hu[i][j] * dK[j];
      s += 2.0 * alpha * t;
    }
    for (int j = 0; j < 3; ++j) s -= 2.0 * Au[i][j] * dalpha[j];
    for (int j = 0; j < 3; ++j)
      s += 2.0 * hu[i][j] * (alpha * dTh[j] - Th * dalpha[j] - (2.0 / 3.0) * alpha * K * Zl[j]);
    s -= 2.0 * alpha * k1 * Zt[i];
    for (int j = 0; j < 3; ++j) s -= 2.0 * alpha * hu[i][j] * S8im[j];
    {
      T t = 0.0;
      for (int j = 0; j < 3; ++j) {
        T AZ = 0.0;
        for (int k = 0; k < 3; ++k) AZ += A[j][k] * Zt[k];
        t += hu[i][j] * (Mi[j] - S8im[j] + dTh[j] - k1 * Zl[j] - AZ - K * Zl[j] / 3.0);
      }
      s -= 2.0 * alpha * fb * t;
    }
    rGam[i] = s;
    r[GH1 + i] = s;
  }
  using std::pow;
  const T apow = (P.lapse_power == 1.0) ? alpha : T(pow(alpha, P.lapse_power));
  // reading: the a-modification divides the lapse source and the B source by (1 + a)
  r[LAPSE] = P.lapse_advec * adv[LAPSE] - P.lapse_coeff * apow * (K - 2.0 * Th) / (1.0 + aa);
  for (int i = 0; i < 3; ++i) {
    T Da = 0.0;  // D^i alpha
    for (int j = 0; j < 3; ++j) Da += chi * hu[i][j] * dalpha[j];
    r[SHIFT1 + i] = P.shift_advec * adv[SHIFT1 + i] + P.shift_gamma_coeff * Bv[i] - (aa / (1.0 + aa)) * alpha * Da;
  }
  for (int i = 0; i < 3; ++i)
    r[BB1 + i] = rGam[i] / (1.0 + aa) - P.eta * Bv[i] +
                 P.shift_advec * (adv[BB1 + i] - adv[GH1 + i] / (1.0 + aa));
  r[PHI] = adv[PHI] + alpha * Pi;
  r[PI_] = adv[PI_] + alpha * ps;

  for (int f = 0; f < NF; ++f)
    if (!finite_val(r[f])) flags |= FLAG_NONFINITE;
  out.ham = Hg - 2.0 * rho8m;
  // the three pieces of 8 pi rho, one per term of the action, divided by 8 pi
  const T inv8pi = 1.0 / (8.0 * M_PI);
  out.rho[0] = (0.5 * Pi * Pi - 0.5 * X) * inv8pi;
  out.rho[1] = g2 * (X * Pi * Pi - 0.5 * X * X) * inv8pi;
  out.rho[2] = H00 * inv8pi;
  // The Gauss-Bonnet invariant as the scalar's row of the system reads it: its
  // spatial part 8 M_i M^i - 4 B_ijk B^ijk plus 8 G^kl C_kl with the solved
  // C_kl.  The weak-coupling indicators (readings; the paper plots where such
  // conditions exceed one without defining them): the Gauss-Bonnet coupling
  // against the curvature scale, |lambda'(phi)| sqrt|L_GB|, and the X^2 term
  // against the X term, |2 g2 X|.
  {
    T gc = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) gc += Gcu[i][j] * Cs[i][j];
    out.lgb = 8.0 * gc + 8.0 * M2 - 4.0 * B2;
    using std::abs;
    using std::sqrt;
    out.weak[0] = abs(dlam) * sqrt(abs(out.lgb));
    out.weak[1] = abs(2.0 * g2 * X);
  }
  for (int i = 0; i < 3; ++i) out.mom[i] = Mi[i] - S8im[i];
  out.flags = flags;
}

// ---------------------------------------------------------------- box level
struct Box {
  int nx, ny, nz;       // interior cells
  int ng;               // ghost layers on every side (3; 4 for the sixth-order scheme with its own dissipation)
  double dx[3];         // spacing along x, y, z
  int64_t sx, sy, sz;   // strides (x is contiguous)
  int64_t fstride;      // elements per field
};

// dims: nx, ny, nz, ghost layers
Box make_box(const int* dims, const double* spacing) {
  Box b;
  b.nx = dims[0];
  b.ny = dims[1];
  b.nz = dims[2];
  b.ng = dims[3];
  for (int d = 0; d < 3; ++d) b.dx[d] = spacing[d];
  b.sx = 1;
  b.sy = b.nx + 2 * b.ng;
  b.sz = int64_t(b.nx + 2 * b.ng) * (b.ny + 2 * b.ng);
  b.fstride = b.sz * (b.nz + 2 * b.ng);
  return b;
}
inline int64_t cell_index(const Box& b, int i, int j, int k) {
  return int64_t(k + b.ng) * b.sz + int64_t(j + b.ng) * b.sy + (i + b.ng);
}

template <class T>
Params<T> read_params(const double* p, const double* pim) {
  Params<T> P;
  P.lambda_gb = p[0];
  P.g2 = p[1];
  P.a = p[2];
  P.b = p[3];
  P.kappa1 = p[4];
  P.kappa2 = p[5];
  P.kappa3 = p[6];
  P.lapse_coeff = p[7];
  P.lapse_power = p[8];
  P.lapse_advec = p[9];
  P.shift_gamma_coeff = p[10];
  P.shift_advec = p[11];
  P.eta = p[12];
  P.ko_sigma = p[13];
  P.decoupled = p[14];
  P.fd_order = (int)p[15];
  P.lambda_lin = p[16];
  P.beta = p[17];
  (void)pim;
  return P;
}
template <>
Params<cplx> read_params<cplx>(const double* p, const double* pim) {
  Params<double> Pd = read_params<double>(p, nullptr);
  Params<cplx> P;
  P.lambda_gb = cplx(p[0], pim ? pim[0] : 0.0);
  P.g2 = cplx(p[1], pim ? pim[1] : 0.0);
  P.a = Pd.a;
  P.b = Pd.b;
  P.kappa1 = Pd.kappa1;
  P.kappa2 = Pd.kappa2;
  P.kappa3 = Pd.kappa3;
  P.lapse_coeff = Pd.lapse_coeff;
  P.lapse_power = Pd.lapse_power;
  P.lapse_advec = Pd.lapse_advec;
  P.shift_gamma_coeff = Pd.shift_gamma_coeff;
  P.shift_advec = Pd.shift_advec;
  P.decoupled = Pd.decoupled;
  P.fd_order = Pd.fd_order;
  P.lambda_lin = Pd.lambda_lin;
  P.beta = Pd.beta;
  P.eta = Pd.eta;
  P.ko_sigma = Pd.ko_sigma;
  return P;
}

// Gather the finite-difference inputs of one cell.  The stencils are the
// 4th-order centred, mixed and lopsided-upwind ones of the cited CCZ4 code
// family; Kreiss-Oliger is the 6th difference with weight sigma/(64 h).
// Sixth-order centred differences on the same three ghost layers:
//   d_k u   = (-u_-3 + 9 u_-2 - 45 u_-1 + 45 u_1 - 9 u_2 + u_3) / (60 h),
//   d_k^2 u = (2 u_-3 - 27 u_-2 + 270 u_-1 - 490 u_0 + 270 u_1 - 27 u_2 + 2 u_3) / (180 h^2),
//   d_k d_l u: the first-derivative weights applied along k and along l (49 points);
// the advection derivative, on a box with three ghost layers, is the
// fifth-order stencil biased one cell towards the side the shift points to
// (offsets -2..3 for beta >= 0, -3..2 otherwise), the widest such stencil
// that three layers hold; with four ghost layers it is the sixth-order
// stencil on offsets -2..4 (beta >= 0) or -4..2,
//   (2 u_-2 - 24 u_-1 - 35 u_0 + 80 u_1 - 30 u_2 + 8 u_3 - u_4) / (60 h),
// which is exact on polynomials of degree 6.
template <class T>
void gather_sixth(const Box& b, const T* u, int64_t c, PointIn<T>& in) {
  const int64_t st[3] = {b.sx, b.sy, b.sz};
  const double w1[7] = {-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0};
  const double w2[7] = {2.0, -27.0, 270.0, -490.0, 270.0, -27.0, 2.0};
  const double wup[6] = {3.0, -30.0, -20.0, 60.0, -15.0, 2.0};          // offsets -2..3, over 60 h
  const double wup7[7] = {2.0, -24.0, -35.0, 80.0, -30.0, 8.0, -1.0};    // offsets -2..4, over 60 h
  for (int f = 0; f < NF; ++f) {
    const T* uf = u + f * b.fstride;
    for (int d = 0; d < 3; ++d) {
      const int64_t s = st[d];
      const double hd = b.dx[d];
      T a1 = 0.0, a2 = 0.0;
      for (int o = -3; o <= 3; ++o) {
        a1 += w1[o + 3] * uf[c + o * s];
        a2 += w2[o + 3] * uf[c + o * s];
      }
      in.d1[f][d] = a1 / (60.0 * hd);
      in.d2[f][SYM[d][d]] = a2 / (180.0 * hd * hd);
    }
    for (int d = 0; d < 3; ++d)
      for (int e = d + 1; e < 3; ++e) {
        T sm = 0.0;
        for (int pa = -3; pa <= 3; ++pa)
          for (int pb = -3; pb <= 3; ++pb) sm += (w1[pa + 3] * w1[pb + 3]) * uf[c + pa * st[d] + pb * st[e]];
        in.d2[f][SYM[d][e]] = sm / (3600.0 * b.dx[d] * b.dx[e]);
      }
  }
  for (int d = 0; d < 3; ++d) {
    const double bsign = re(in.u[SHIFT1 + d]);
    const int64_t s = st[d];
    const double hd = b.dx[d];
    for (int f = 0; f < NF; ++f) {
      const T* uf = u + f * b.fstride;
      T a = 0.0;
      // beta >= 0: offsets -2..3 (-2..4); beta < 0: the mirror image with the sign flipped
      if (b.ng >= 4)
        for (int q = 0; q < 7; ++q) a += bsign >= 0.0 ? wup7[q] * uf[c + (q - 2) * s] : -wup7[q] * uf[c - (q - 2) * s];
      else
        for (int q = 0; q < 6; ++q) a += bsign >= 0.0 ? wup[q] * uf[c + (q - 2) * s] : -wup[q] * uf[c - (q - 2) * s];
      in.adv[f][d] = a / (60.0 * hd);
    }
  }
}

template <class T>
void gather_point(const Box& b, const T* u, int i, int j, int k, PointIn<T>& in, T ko[NF], int order = 4) {
  const int64_t c = cell_index(b, i, j, k);
  const int64_t st[3] = {b.sx, b.sy, b.sz};
  const double cfd[5] = {1.0, -8.0, 0.0, 8.0, -1.0};  // first-derivative weights at -2..2
  for (int f = 0; f < NF; ++f) {
    const T* uf = u + f * b.fstride;
    in.u[f] = uf[c];
  }
  if (order == 6) {
    gather_sixth(b, u, c, in);
  } else {
  for (int f = 0; f < NF; ++f) {
    const T* uf = u + f * b.fstride;
    for (int d = 0; d < 3; ++d) {
      const int64_t s = st[d];
      const double hd = b.dx[d];
      in.d1[f][d] = (uf[c - 2 * s] - 8.0 * uf[c - s] + 8.0 * uf[c + s] - uf[c + 2 * s]) / (12.0 * hd);
      in.d2[f][SYM[d][d]] = (-uf[c - 2 * s] + 16.0 * uf[c - s] - 30.0 * uf[c] + 16.0 * uf[c + s] - uf[c + 2 * s]) /
                            (12.0 * hd * hd);
    }
    for (int d = 0; d < 3; ++d)
      for (int e = d + 1; e < 3; ++e) {
        T s = 0.0;
        for (int pa = -2; pa <= 2; ++pa)
          for (int pb = -2; pb <= 2; ++pb) {
            const double w = cfd[pa + 2] * cfd[pb + 2];
            if (w == 0.0) continue;
            s += w * uf[c + pa * st[d] + pb * st[e]];
          }
        in.d2[f][SYM[d][e]] = s / (144.0 * b.dx[d] * b.dx[e]);
      }
  }
  // upwinded derivatives, side chosen by the sign of the shift component
  for (int d = 0; d < 3; ++d) {
    const double bsign = re(in.u[SHIFT1 + d]);
    const int64_t s = st[d];
    const double hd = b.dx[d];
    for (int f = 0; f < NF; ++f) {
      const T* uf = u + f * b.fstride;
      if (bsign >= 0.0)
        in.adv[f][d] = (-3.0 * uf[c - s] - 10.0 * uf[c] + 18.0 * uf[c + s] - 6.0 * uf[c + 2 * s] + uf[c + 3 * s]) /
                       (12.0 * hd);
      else
        in.adv[f][d] = (3.0 * uf[c + s] + 10.0 * uf[c] - 18.0 * uf[c - s] + 6.0 * uf[c - 2 * s] - uf[c - 3 * s]) /
                       (12.0 * hd);
    }
  }
  }  // order 4
  // Kreiss-Oliger: with four ghost layers and the sixth-order scheme, minus
  // the eighth difference over 256 h (an O(h^7) term, below the scheme's
  // truncation error); otherwise the sixth difference over 64 h.  Either
  // multiplies the highest grid mode by -1/h.
  const bool ko8 = order == 6 && b.ng >= 4;
  for (int f = 0; f < NF; ++f) {
    const T* uf = u + f * b.fstride;
    T s = 0.0;
    for (int d = 0; d < 3; ++d) {
      const int64_t q = st[d];
      if (ko8) {
        T eight = uf[c - 4 * q] - 8.0 * uf[c - 3 * q] + 28.0 * uf[c - 2 * q] - 56.0 * uf[c - q] + 70.0 * uf[c] -
                  56.0 * uf[c + q] + 28.0 * uf[c + 2 * q] - 8.0 * uf[c + 3 * q] + uf[c + 4 * q];
        s += -eight / (256.0 * b.dx[d]);
      } else {
        T six = uf[c - 3 * q] - 6.0 * uf[c - 2 * q] + 15.0 * uf[c - q] - 20.0 * uf[c] + 15.0 * uf[c + q] -
                6.0 * uf[c + 2 * q] + uf[c + 3 * q];
        s += six / (64.0 * b.dx[d]);
      }
    }
    ko[f] = s;
  }
}

template <class T>
int box_rhs(const Params<T>& P, const Box& b, const T* u, T* rhs, T* ham, T* mom, T* rho = nullptr,
            T* coupling = nullptr) {
  int flags_all = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : flags_all)
  for (int k = 0; k < b.nz; ++k) {
    PointIn<T> in;
    PointOut<T> out;
    T ko[NF];
    for (int j = 0; j < b.ny; ++j)
      for (int i = 0; i < b.nx; ++i) {
        gather_point(b, u, i, j, k, in, ko, P.fd_order);
        rhs_point(P, in, out);
        const int64_t c = cell_index(b, i, j, k);
        if (rhs)
          for (int f = 0; f < NF; ++f) rhs[f * b.fstride + c] = out.rhs[f] + P.ko_sigma * ko[f];
        if (ham) ham[c] = out.ham;
        if (mom)
          for (int d = 0; d < 3; ++d) mom[d * b.fstride + c] = out.mom[d];
        if (rho)
          for (int d = 0; d < 3; ++d) rho[d * b.fstride + c] = out.rho[d];
        if (coupling) {
          coupling[c] = out.lgb;
          coupling[b.fstride + c] = out.weak[0];
          coupling[2 * b.fstride + c] = out.weak[1];
          coupling[3 * b.fstride + c] = out.detA;
        }
        flags_all |= out.flags;
      }
  }
  return flags_all;
}

// periodic ghost fill: every ghost takes the value of the interior cell that is
// congruent to it modulo the box size
template <class T>
void fill_periodic(const Box& b, T* u) {
  const int n[3] = {b.nx, b.ny, b.nz};
#pragma omp parallel for
  for (int k = -b.ng; k < b.nz + b.ng; ++k)
    for (int j = -b.ng; j < b.ny + b.ng; ++j)
      for (int i = -b.ng; i < b.nx + b.ng; ++i) {
        if (i >= 0 && i < n[0] && j >= 0 && j < n[1] && k >= 0 && k < n[2]) continue;
        const int si = ((i % n[0]) + n[0]) % n[0];
        const int sj = ((j % n[1]) + n[1]) % n[1];
        const int sk = ((k % n[2]) + n[2]) % n[2];
        const int64_t dst = cell_index(b, i, j, k), src = cell_index(b, si, sj, sk);
        for (int f = 0; f < NF; ++f) u[f * b.fstride + dst] = u[f * b.fstride + src];
      }
}

// classic RK4 with (c2, c3, c4) = (1/2, 1/2, 1) and weights (1, 2, 2, 1)/6
template <class T>
int rk4_steps(const Params<T>& P, const Box& b, int bc_periodic, double dt, int nsteps, T* u) {
  const int64_t ntot = b.fstride * NF;
  std::vector<T> k1(ntot), k2(ntot), k3(ntot), k4(ntot), us(ntot);
  int flags = 0;
  for (int step = 0; step < nsteps; ++step) {
    auto stage_state = [&](const std::vector<T>& kk, double c) {
      for (int64_t q = 0; q < ntot; ++q) us[q] = u[q];  // ghosts stay at u (frozen) or are refilled
      for (int f = 0; f < NF; ++f)
        for (int kz = 0; kz < b.nz; ++kz)
          for (int jy = 0; jy < b.ny; ++jy)
            for (int ix = 0; ix < b.nx; ++ix) {
              const int64_t q = f * b.fstride + cell_index(b, ix, jy, kz);
              us[q] = u[q] + c * dt * kk[q];
            }
      if (bc_periodic) fill_periodic(b, us.data());
    };
    flags |= box_rhs(P, b, u, k1.data(), (T*)nullptr, (T*)nullptr);
    stage_state(k1, 0.5);
    flags |= box_rhs(P, b, us.data(), k2.data(), (T*)nullptr, (T*)nullptr);
    stage_state(k2, 0.5);
    flags |= box_rhs(P, b, us.data(), k3.data(), (T*)nullptr, (T*)nullptr);
    stage_state(k3, 1.0);
    flags |= box_rhs(P, b, us.data(), k4.data(), (T*)nullptr, (T*)nullptr);
    for (int f = 0; f < NF; ++f)
      for (int kz = 0; kz < b.nz; ++kz)
        for (int jy = 0; jy < b.ny; ++jy)
          for (int ix = 0; ix < b.nx; ++ix) {
            const int64_t q = f * b.fstride + cell_index(b, ix, jy, kz);
            u[q] = u[q] + (dt / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
          }
    if (bc_periodic) fill_periodic(b, u);
  }
  return flags;
}

// ---------------------------------------------------------------- boundary rules
// Key features, "Boundary Conditions": extrapolating, Sommerfeld (radiative),
// reflective and periodic faces.  Faces are numbered x-, x+, y-, y+, z-, z+.
// Every ghost cell belongs to exactly one face: the x face when its x index is
// outside the interior, else the y face when its y index is, else the z face.
// Frozen and Sommerfeld ghosts are evolved by the RK4 step (right-hand side 0
// and the radiative right-hand side respectively); periodic, reflective and
// extrapolating ghosts are refilled from the new state after every stage, the
// z faces first, then y, then x, so that each face reads finished cells only.
enum { FACE_FROZEN = 0, FACE_PERIODIC = 1, FACE_REFLECTIVE = 2, FACE_EXTRAPOLATING = 3, FACE_SOMMERFELD = 4 };

struct BcSpec {
  int rule[6];
  int extrap_order;      // 0: copy the boundary cell, 1: linear through the two outermost interior cells
  double origin[3];      // coordinates of the centre of interior cell (0, 0, 0)
  double centre[3];      // centre of the radiative condition
  double speed[NF];      // radiative speed per field
  double asymptote[NF];  // value at infinity per field
  int parity_phi;        // sign of phi and Pi under a reflection
};

// packed as doubles: rule[6], extrap_order, origin[3], centre[3], speed[27], asymptote[27], parity_phi
BcSpec read_bc(const double* v) {
  BcSpec s;
  int q = 0;
  for (int f = 0; f < 6; ++f) s.rule[f] = (int)v[q++];
  s.extrap_order = (int)v[q++];
  for (int d = 0; d < 3; ++d) s.origin[d] = v[q++];
  for (int d = 0; d < 3; ++d) s.centre[d] = v[q++];
  for (int f = 0; f < NF; ++f) s.speed[f] = v[q++];
  for (int f = 0; f < NF; ++f) s.asymptote[f] = v[q++];
  s.parity_phi = (int)v[q++];
  return s;
}

// face owning cell (i, j, k), -1 for an interior cell
int owner_face(const Box& b, int i, int j, int k) {
  if (i < 0) return 0;
  if (i >= b.nx) return 1;
  if (j < 0) return 2;
  if (j >= b.ny) return 3;
  if (k < 0) return 4;
  if (k >= b.nz) return 5;
  return -1;
}

// Sign of field f under the reflection x_axis -> -x_axis: one factor -1 per
// tensor index of the field along that axis (h_ij and A_ij two indices,
// Gamma^i, beta^i and B^i one); the scalar and its momentum take parity_phi.
int field_parity(int f, int axis, int parity_phi) {
  if (f == PHI || f == PI_) return parity_phi;
  int count = 0;
  auto sym_pair = [&](int base) {
    for (int a = 0; a < 3; ++a)
      for (int c = a; c < 3; ++c)
        if (f == base + SYM[a][c]) count = (a == axis) + (c == axis);
  };
  if (f >= H11 && f < H11 + 6) sym_pair(H11);
  if (f >= A11 && f < A11 + 6) sym_pair(A11);
  if (f >= GH1 && f < GH1 + 3) count = (f - GH1 == axis);
  if (f >= SHIFT1 && f < SHIFT1 + 3) count = (f - SHIFT1 == axis);
  if (f >= BB1 && f < BB1 + 3) count = (f - BB1 == axis);
  return (count % 2) ? -1 : 1;
}

template <class T>
void fill_faces(const Box& b, const BcSpec& bc, T* u) {
  const int n[3] = {b.nx, b.ny, b.nz};
  for (int axis = 2; axis >= 0; --axis) {
    for (int k = -b.ng; k < b.nz + b.ng; ++k)
      for (int j = -b.ng; j < b.ny + b.ng; ++j)
        for (int i = -b.ng; i < b.nx + b.ng; ++i) {
          const int face = owner_face(b, i, j, k);
          if (face < 0 || face / 2 != axis) continue;
          const int rule = bc.rule[face];
          if (rule != FACE_PERIODIC && rule != FACE_REFLECTIVE && rule != FACE_EXTRAPOLATING) continue;
          int idx[3] = {i, j, k};
          const int m = idx[axis], na = n[axis];
          const bool low = m < 0;
          auto at = [&](int f, int mm) {
            int q[3] = {idx[0], idx[1], idx[2]};
            q[axis] = mm;
            return u[f * b.fstride + cell_index(b, q[0], q[1], q[2])];
          };
          const int64_t dst = cell_index(b, i, j, k);
          for (int f = 0; f < NF; ++f) {
            T v;
            if (rule == FACE_PERIODIC) {
              v = at(f, ((m % na) + na) % na);
            } else if (rule == FACE_REFLECTIVE) {
              v = T(field_parity(f, axis, bc.parity_phi)) * at(f, low ? -1 - m : 2 * na - 1 - m);
            } else {
              const int e = low ? 0 : na - 1;      // outermost interior cell
              const int e2 = low ? 1 : na - 2;     // its interior neighbour
              const T ue = at(f, e);
              v = bc.extrap_order == 0 ? ue : ue + T(double(std::abs(m - e))) * (ue - at(f, e2));
            }
            u[f * b.fstride + dst] = v;
          }
        }
  }
}

// Radiative right-hand side of field f at ghost cell (i, j, k):
//   d_t f = -v (x^a d_a f) / r - v (f - f_inf) / r,   x^a relative to the centre,
// with second-order differences: one-sided towards the interior along the axes
// on which the cell lies outside the interior, centred along the others.
template <class T>
T sommerfeld_rhs(const Box& b, const BcSpec& bc, const T* u, int f, int i, int j, int k) {
  const int n[3] = {b.nx, b.ny, b.nz};
  const int idx[3] = {i, j, k};
  const T* uf = u + f * b.fstride;
  auto at = [&](int axis, int off) {
    int q[3] = {i, j, k};
    q[axis] += off;
    return uf[cell_index(b, q[0], q[1], q[2])];
  };
  double x[3];
  double r2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    x[a] = bc.origin[a] + idx[a] * b.dx[a] - bc.centre[a];
    r2 += x[a] * x[a];
  }
  const double r = std::sqrt(r2);
  T xdf = 0.0;
  for (int a = 0; a < 3; ++a) {
    T d;
    if (idx[a] < 0)
      d = (-3.0 * at(a, 0) + 4.0 * at(a, 1) - at(a, 2)) / (2.0 * b.dx[a]);
    else if (idx[a] >= n[a])
      d = (3.0 * at(a, 0) - 4.0 * at(a, -1) + at(a, -2)) / (2.0 * b.dx[a]);
    else
      d = (at(a, 1) - at(a, -1)) / (2.0 * b.dx[a]);
    xdf += x[a] * d;
  }
  const T fv = at(0, 0);
  return -bc.speed[f] * xdf / r - bc.speed[f] * (fv - bc.asymptote[f]) / r;
}

// right-hand side in the ghost cells: radiative on Sommerfeld faces, 0 elsewhere
template <class T>
void ghost_rhs(const Box& b, const BcSpec& bc, const T* u, T* rhs) {
  for (int k = -b.ng; k < b.nz + b.ng; ++k)
    for (int j = -b.ng; j < b.ny + b.ng; ++j)
      for (int i = -b.ng; i < b.nx + b.ng; ++i) {
        const int face = owner_face(b, i, j, k);
        if (face < 0) continue;
        const int64_t c = cell_index(b, i, j, k);
        for (int f = 0; f < NF; ++f)
          rhs[f * b.fstride + c] = bc.rule[face] == FACE_SOMMERFELD ? sommerfeld_rhs(b, bc, u, f, i, j, k) : T(0.0);
      }
}

// classic RK4 over interior and ghost cells with the face rules above
template <class T>
int rk4_steps_bc(const Params<T>& P, const Box& b, const BcSpec& bc, double dt, int nsteps, T* u) {
  const int64_t ntot = b.fstride * NF;
  std::vector<T> k1(ntot), k2(ntot), k3(ntot), k4(ntot), us(ntot);
  int flags = 0;
  auto rhs_all = [&](const T* v, std::vector<T>& kk) {
    flags |= box_rhs(P, b, v, kk.data(), (T*)nullptr, (T*)nullptr);
    ghost_rhs(b, bc, v, kk.data());
  };
  for (int step = 0; step < nsteps; ++step) {
    auto stage_state = [&](const std::vector<T>& kk, double c) {
      for (int64_t q = 0; q < ntot; ++q) us[q] = u[q] + c * dt * kk[q];
      fill_faces(b, bc, us.data());
    };
    rhs_all(u, k1);
    stage_state(k1, 0.5);
    rhs_all(us.data(), k2);
    stage_state(k2, 0.5);
    rhs_all(us.data(), k3);
    stage_state(k3, 1.0);
    rhs_all(us.data(), k4);
    for (int64_t q = 0; q < ntot; ++q) u[q] = u[q] + (dt / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    fill_faces(b, bc, u);
  }
  return flags;
}

}  // namespace

// ---------------------------------------------------------------- C ABI
// Parameter array (18 doubles): lambda_gb, g2, a, b, kappa1, kappa2, kappa3,
// lapse_coeff, lapse_power, lapse_advec, shift_gamma_coeff, shift_advec, eta, ko_sigma,
// decoupled, fd_order, lambda_lin, beta.
extern "C" {

int oracle_nfields() { return NF; }

// Full-box right-hand side on interior cells (rhs ghosts untouched).  Returns OR of cell flags.
int oracle_rhs(const double* params, const int* dims, const double* spacing, const double* u, double* rhs) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  return box_rhs(P, b, u, rhs, (double*)nullptr, (double*)nullptr);
}

// Right-hand side at a list of interior cells (i, j, k triples); out is [ncell][27].
int oracle_rhs_cells(const double* params, const int* dims, const double* spacing, const double* u, int ncell,
                     const int* ijk, double* out) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  int flags_all = 0;
#pragma omp parallel for reduction(| : flags_all)
  for (int q = 0; q < ncell; ++q) {
    PointIn<double> in;
    PointOut<double> o;
    double ko[NF];
    gather_point(b, u, ijk[3 * q], ijk[3 * q + 1], ijk[3 * q + 2], in, ko, P.fd_order);
    rhs_point(P, in, o);
    for (int f = 0; f < NF; ++f) out[q * NF + f] = o.rhs[f] + P.ko_sigma * ko[f];
    flags_all |= o.flags;
  }
  return flags_all;
}

// Complex-step right-hand side: state u + i*u_im, couplings theta + i*theta_im.
int oracle_rhs_cs(const double* params, const double* theta_im, const int* dims, const double* spacing,
                  const double* u_re, const double* u_im, double* rhs_re, double* rhs_im) {
  Box b = make_box(dims, spacing);
  Params<cplx> P = read_params<cplx>(params, theta_im);
  const int64_t n = b.fstride * NF;
  std::vector<cplx> u(n), r(n, cplx(0.0, 0.0));
  for (int64_t q = 0; q < n; ++q) u[q] = cplx(u_re[q], u_im ? u_im[q] : 0.0);
  int fl = box_rhs(P, b, u.data(), r.data(), (cplx*)nullptr, (cplx*)nullptr);
  for (int64_t q = 0; q < n; ++q) {
    rhs_re[q] = r[q].real();
    rhs_im[q] = r[q].imag();
  }
  return fl;
}

// Hamiltonian and momentum constraints on interior cells (ham: one field, mom: three).
int oracle_constraints(const double* params, const int* dims, const double* spacing, const double* u, double* ham,
                       double* mom) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  return box_rhs(P, b, u, (double*)nullptr, ham, mom);
}

// Energy densities of the canonical, X^2 and Gauss-Bonnet terms on interior cells (rho: three fields).
int oracle_energy_densities(const double* params, const int* dims, const double* spacing, const double* u,
                            double* rho) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  return box_rhs(P, b, u, (double*)nullptr, (double*)nullptr, (double*)nullptr, rho);
}

// Fill the ghosts of periodic, reflective and extrapolating faces (bc packed as above).
void oracle_fill_bc(const int* dims, const double* spacing, const double* bcv, double* u) {
  Box b = make_box(dims, spacing);
  fill_faces(b, read_bc(bcv), u);
}

// Ghost right-hand side (radiative on Sommerfeld faces, 0 on other ghosts); interior of rhs untouched.
void oracle_ghost_rhs(const int* dims, const double* spacing, const double* bcv, const double* u, double* rhs) {
  Box b = make_box(dims, spacing);
  ghost_rhs(b, read_bc(bcv), u, rhs);
}

// nsteps RK4 steps in place with per-face boundary rules.
int oracle_rk4_bc(const double* params, const int* dims, const double* spacing, const double* bcv, double dt,
                  int nsteps, double* u) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  return rk4_steps_bc(P, b, read_bc(bcv), dt, nsteps, u);
}

// Gauss-Bonnet invariant, the two weak-coupling indicators and the determinant of the
// per-cell system on interior cells (four fields).
int oracle_coupling(const double* params, const int* dims, const double* spacing, const double* u, double* out) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  return box_rhs(P, b, u, (double*)nullptr, (double*)nullptr, (double*)nullptr, (double*)nullptr, out);
}

void oracle_fill_periodic(const int* dims, double* u) {
  const double sp[3] = {1.0, 1.0, 1.0};
  Box b = make_box(dims, sp);
  fill_periodic(b, u);
}

// nsteps RK4 steps in place.  bc: 0 frozen ghosts, 1 periodic.
// Algorithmic flops per interior cell (the convention of the Flop type above),
// counted by running this file's own code on Flop values: the state u (state
// layout, ghosts filled) and the two couplings variable, everything else
// constant.  Single-threaded while counting.
//   out[0]  one right-hand side (Kreiss-Oliger included) at an interior cell,
//           mean over the interior cells;
//   out[1]  the part of out[0] in the stencils and the Kreiss-Oliger sum;
//   out[2]  one classic RK4 step per interior cell (four right-hand sides and
//           the stage updates), the box taken as periodic.
int oracle_flops_per_cell(const double* params, const int* dims, const double* spacing, const double* u,
                          double* out) {
  Box b = make_box(dims, spacing);
  Params<double> Pd = read_params<double>(params, nullptr);
  Params<Flop> P;
  P.lambda_gb = Flop::var(Pd.lambda_gb);
  P.g2 = Flop::var(Pd.g2);
  P.a = Pd.a;
  P.b = Pd.b;
  P.kappa1 = Pd.kappa1;
  P.kappa2 = Pd.kappa2;
  P.kappa3 = Pd.kappa3;
  P.lapse_coeff = Pd.lapse_coeff;
  P.lapse_power = Pd.lapse_power;
  P.lapse_advec = Pd.lapse_advec;
  P.shift_gamma_coeff = Pd.shift_gamma_coeff;
  P.shift_advec = Pd.shift_advec;
  P.eta = Pd.eta;
  P.ko_sigma = Pd.ko_sigma;
  P.decoupled = Pd.decoupled;
  P.fd_order = Pd.fd_order;
  P.lambda_lin = Pd.lambda_lin;
  P.beta = Pd.beta;
  const int64_t ntot = b.fstride * NF;
  std::vector<Flop> uf(ntot);
  for (int64_t q = 0; q < ntot; ++q) uf[q] = Flop::var(u[q]);
  const int keep = omp_get_max_threads();
  omp_set_num_threads(1);
  const int64_t ncell = (int64_t)b.nx * b.ny * b.nz;
  int64_t rhs_ops = 0, gather_ops = 0;
  int flags = 0;
  for (int k = 0; k < b.nz; ++k)
    for (int j = 0; j < b.ny; ++j)
      for (int i = 0; i < b.nx; ++i) {
        PointIn<Flop> in;
        PointOut<Flop> o;
        Flop ko[NF];
        g_tape.clear();
        gather_point(b, uf.data(), i, j, k, in, ko, P.fd_order);
        const int32_t gathered = (int32_t)g_tape.size();
        rhs_point(P, in, o);
        std::vector<int32_t> outs;
        for (int f = 0; f < NF; ++f) outs.push_back((o.rhs[f] + P.ko_sigma * ko[f]).id);
        // the stencil part: live operations recorded by the gather
        std::vector<char> live(g_tape.size(), 0);
        for (int32_t q : outs)
          if (q >= 0) live[q] = 1;
        for (int64_t q = (int64_t)g_tape.size() - 1; q >= 0; --q) {
          if (!live[q]) continue;
          ++rhs_ops;
          if (q < gathered) ++gather_ops;
          if (g_tape[q].a >= 0) live[g_tape[q].a] = 1;
          if (g_tape[q].b >= 0) live[g_tape[q].b] = 1;
        }
        flags |= o.flags;
      }
  g_tape.clear();
  flags |= rk4_steps(P, b, 1, 0.01, 1, uf.data());
  std::vector<int32_t> outs;
  for (int f = 0; f < NF; ++f)
    for (int k = 0; k < b.nz; ++k)
      for (int j = 0; j < b.ny; ++j)
        for (int i = 0; i < b.nx; ++i) outs.push_back(uf[f * b.fstride + cell_index(b, i, j, k)].id);
  const int64_t step_ops = flop_count_live(outs);
  g_tape.clear();
  g_tape.shrink_to_fit();
  omp_set_num_threads(keep);
  out[0] = double(rhs_ops) / double(ncell);
  out[1] = double(gather_ops) / double(ncell);
  out[2] = double(step_ops) / double(ncell);
  return flags;
}

// The same RK4 steps carried out in long double throughout (state, stencils,
// algebra, the per-cell solve); u is read and the result written back rounded
// to double.
int oracle_rk4_ld(const double* params, const int* dims, const double* spacing, int bc, double dt, int nsteps,
                  double* u) {
  Box b = make_box(dims, spacing);
  Params<long double> P = read_params<long double>(params, nullptr);
  const int64_t ntot = b.fstride * NF;
  std::vector<long double> ul(u, u + ntot);
  const int flags = rk4_steps(P, b, bc, (long double)dt, nsteps, ul.data());
  for (int64_t q = 0; q < ntot; ++q) u[q] = (double)ul[q];
  return flags;
}

int oracle_rk4(const double* params, const int* dims, const double* spacing, int bc, double dt, int nsteps,
               double* u) {
  Box b = make_box(dims, spacing);
  Params<double> P = read_params<double>(params, nullptr);
  return rk4_steps(P, b, bc, dt, nsteps, u);
}

// Complex-step RK4: advances u_re + i u_im with couplings theta + i theta_im.
int oracle_rk4_cs(const double* params, const double* theta_im, const int* dims, const double* spacing, int bc,
                  double dt, int nsteps, double* u_re, double* u_im) {
  Box b = make_box(dims, spacing);
  Params<cplx> P = read_params<cplx>(params, theta_im);
  const int64_t n = b.fstride * NF;
  std::vector<cplx> u(n);
  for (int64_t q = 0; q < n; ++q) u[q] = cplx(u_re[q], u_im[q]);
  int fl = rk4_steps(P, b, bc, dt, nsteps, u.data());
  for (int64_t q = 0; q < n; ++q) {
    u_re[q] = u[q].real();
    u_im[q] = u[q].imag();
  }
  return fl;
}

// Pointwise right-hand side from given values and derivatives (no stencils,
// no Kreiss-Oliger).  d1: [27][3], d2: [27][6] packed (xx,xy,xz,yy,yz,zz),
// adv: [27][3].  extra (may be null) receives
//   ham, mom[3], C[6], p, sysA[49], sysb[7], pivot_ratio  (68 doubles).
int oracle_rhs_point(const double* params, const double* u, const double* d1, const double* d2, const double* adv,
                     double* rhs, double* extra) {
  Params<double> P = read_params<double>(params, nullptr);
  PointIn<double> in;
  PointOut<double> o;
  for (int f = 0; f < NF; ++f) {
    in.u[f] = u[f];
    for (int d = 0; d < 3; ++d) {
      in.d1[f][d] = d1[f * 3 + d];
      in.adv[f][d] = adv[f * 3 + d];
    }
    for (int d = 0; d < 6; ++d) in.d2[f][d] = d2[f * 6 + d];
  }
  rhs_point(P, in, o);
  for (int f = 0; f < NF; ++f) rhs[f] = o.rhs[f];
  if (extra) {
    int q = 0;
    extra[q++] = o.ham;
    for (int d = 0; d < 3; ++d) extra[q++] = o.mom[d];
    for (int d = 0; d < 6; ++d) extra[q++] = o.C[d];
    extra[q++] = o.p;
    for (int d = 0; d < 49; ++d) extra[q++] = o.sysA[d];
    for (int d = 0; d < 7; ++d) extra[q++] = o.sysb[d];
    extra[q++] = o.pivot_ratio;
    for (int d = 0; d < 3; ++d) extra[q++] = o.rho[d];
    extra[q++] = o.lgb;
    extra[q++] = o.weak[0];
    extra[q++] = o.weak[1];
    extra[q++] = o.detA;
  }
  return o.flags;
}

// Post-stage algebraic enforcement (interior cells, in place): the conformal
// metric is rescaled to unit determinant, A_ij loses its trace with respect to
// the rescaled metric, chi and the lapse are floored.
void oracle_enforce(const int* dims, double* u, double chi_min, double lapse_min) {
  const double sp[3] = {1.0, 1.0, 1.0};
  Box b = make_box(dims, sp);
  for (int k = 0; k < b.nz; ++k)
    for (int j = 0; j < b.ny; ++j)
      for (int i = 0; i < b.nx; ++i) {
        const int64_t c = cell_index(b, i, j, k);
        double h[3][3], A[3][3], hu[3][3];
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) {
            h[a][bb] = u[(H11 + SYM[a][bb]) * b.fstride + c];
            A[a][bb] = u[(A11 + SYM[a][bb]) * b.fstride + c];
          }
        const double scale = 1.0 / std::cbrt(det3(h));
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) h[a][bb] *= scale;
        inv3(h, hu);
        double tr = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) tr += hu[a][bb] * A[a][bb];
        for (int a = 0; a < 3; ++a)
          for (int bb = a; bb < 3; ++bb) {
            u[(H11 + SYM[a][bb]) * b.fstride + c] = h[a][bb];
            u[(A11 + SYM[a][bb]) * b.fstride + c] = A[a][bb] - h[a][bb] * tr / 3.0;
          }
        if (u[CHI * b.fstride + c] < chi_min) u[CHI * b.fstride + c] = chi_min;
        if (u[LAPSE * b.fstride + c] < lapse_min) u[LAPSE * b.fstride + c] = lapse_min;
      }
}

// The oracle's dense solver, exposed for checking against a library solve.
double oracle_gepp(int n, const double* A, const double* b, double* x) {
  std::vector<double> Aw(A, A + n * n), bw(b, b + n);
  return gepp_solve(n, Aw.data(), bw.data(), x);
}

// Finite-difference stencils of one scalar field at one cell, for polynomial pins.
// out: d1[3], d2[6], adv_plus[3], adv_minus[3], ko (one value, sigma = 1)  -> 16 doubles
void oracle_stencils(const int* dims, const double* spacing, const double* f, int i, int j, int k, int order,
                     double* out) {
  Box b = make_box(dims, spacing);
  // place the scalar in field 0 of a scratch state; the shift sign selects the upwind side
  std::vector<double> u(b.fstride * NF, 0.0);
  std::memcpy(u.data(), f, sizeof(double) * b.fstride);
  PointIn<double> in;
  double ko[NF];
  const int64_t c = cell_index(b, i, j, k);
  for (int d = 0; d < 3; ++d) u[(SHIFT1 + d) * b.fstride + c] = 1.0;
  gather_point(b, u.data(), i, j, k, in, ko, order);
  int q = 0;
  for (int d = 0; d < 3; ++d) out[q++] = in.d1[0][d];
  for (int d = 0; d < 6; ++d) out[q++] = in.d2[0][d];
  for (int d = 0; d < 3; ++d) out[q++] = in.adv[0][d];
  for (int d = 0; d < 3; ++d) u[(SHIFT1 + d) * b.fstride + c] = -1.0;
  gather_point(b, u.data(), i, j, k, in, ko, order);
  for (int d = 0; d < 3; ++d) out[q++] = in.adv[0][d];
  out[q++] = ko[0];
}

}  // extern "C"
