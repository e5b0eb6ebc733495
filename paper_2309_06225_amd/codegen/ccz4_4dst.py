"""Pointwise 4dST + modified-CCZ4 right-hand side as an expression graph.

The equations (the paper prints none; they are the 3+1 form of the 4dST theory
with backreaction that the paper's Summary and Key features name):
  * theory: (1/16pi) sqrt(-g) [R + X + lambda(phi) L_GB + g2 X^2],
    X = -1/2 (d phi)^2, lambda = lambda_gb phi^2/4, V = 0;
  * CCZ4 (kappa1, kappa2, kappa3) with the Z4 trace reversal taken with
    hat g = g - b n n, and the modified puncture gauge with a;
  * the Gauss-Bonnet stress is affine in C_ij = 4R_{injn} and p = Lie_n Pi,
    which are found from a 7x7 linear system per cell.

Inputs of the graph (per cell): the 27 field values, centred first derivatives
of the 24 fields that need them, centred second derivatives of 12 fields, and
the upwinded advection sums beta^k d_k u for the advected fields.  Outputs:
the 27 right-hand sides without Kreiss-Oliger dissipation (added by the
kernel), plus the pivots of the elimination (for the hyperbolicity flag).
"""
from __future__ import annotations

import math

from .expr import Graph, Node

NF = 27
CHI, H0, K_, A0, THETA, GH0, LAPSE, SHIFT0, BB0, PHI, PI = 0, 1, 7, 8, 14, 15, 18, 19, 22, 25, 26
# fields whose centred first derivatives are used (all but B^i)
D1_FIELDS = [f for f in range(NF) if not (BB0 <= f < BB0 + 3)]
# fields whose second derivatives are used: chi, h_ij, lapse, shift, phi
D2_FIELDS = [CHI] + list(range(H0, H0 + 6)) + [LAPSE] + list(range(SHIFT0, SHIFT0 + 3)) + [PHI]
SYM6 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
PACK = [[0, 1, 2], [1, 3, 4], [2, 4, 5]]
# advected fields; the shift and B only when shift advection is on
ADV_ALWAYS = [f for f in range(NF) if not (SHIFT0 <= f < BB0 + 3)]
ADV_SHIFT = list(range(SHIFT0, BB0 + 3))


def merged_adv(shift_advec: bool):
    """Fields whose advection sum enters only their own right-hand side, with
    coefficient 1: all advected fields but the lapse (coefficient lapse_advec)
    and Gamma^i (its right-hand side, advection included, also drives B^i).
    The stencil stage adds their sum to the field's Kreiss-Oliger term, so the
    pointwise algebra never reads it."""
    del shift_advec  # the same set with and without shift advection
    return [f for f in ADV_ALWAYS if f != LAPSE and not (GH0 <= f < GH0 + 3)]

PARAMS = ("lambda_gb", "g2", "kappa1", "kappa3", "k1_1pk2", "k1_2pk2", "k1k2",
          "lapse_coeff", "lapse_advec", "shift_gamma_coeff", "shift_advec", "eta",
          "inv1pa", "a_1pa", "fb", "cfac", "b4", "lambda_lin", "beta")


def _eps(a, b, c):
    if len({a, b, c}) < 3:
        return 0
    return 1 if (a, b, c) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1


def input_names(shift_advec: bool):
    names = [f"u{f}" for f in range(NF)]
    names += [f"d1_{f}_{k}" for f in D1_FIELDS for k in range(3)]
    names += [f"d2_{f}_{q}" for f in D2_FIELDS for q in range(6)]
    names += [f"adv{f}" for f in (ADV_ALWAYS + (ADV_SHIFT if shift_advec else []))
              if f not in merged_adv(shift_advec)]
    return names


def build(shift_advec: bool = False, decoupled: bool = False, general_coupling: bool = True):
    """decoupled: the decoupling limit of 4dST (the scalar moves on the metric
    without sourcing it): the metric equations see no energy, momentum,
    stress or Gauss-Bonnet tensor and their rows of the per-cell system reduce
    to C_ij = Q_ij; the scalar's row is unchanged.  general_coupling:
    lambda(phi) = lambda_lin phi + lambda_gb (1 - exp(-beta phi^2))/(4 beta)
    (beta = 0: lambda_gb phi^2 / 4); without it the graph is the purely
    quadratic coupling's, for the default staged kernel."""
    g = Graph()
    S = g.sum
    P = {n: g.param(n) for n in PARAMS}
    u = [g.input(f"u{f}") for f in range(NF)]
    d1 = {f: [g.input(f"d1_{f}_{k}") for k in range(3)] for f in D1_FIELDS}
    d2 = {f: [[g.input(f"d2_{f}_{PACK[k][l]}") for l in range(3)] for k in range(3)] for f in D2_FIELDS}
    adv_fields = ADV_ALWAYS + (ADV_SHIFT if shift_advec else [])
    merged = merged_adv(shift_advec)
    adv = {f: g.input(f"adv{f}") for f in adv_fields if f not in merged}
    zero = g.const(0.0)

    def sym(vals):
        return [[vals[PACK[i][j]] for j in range(3)] for i in range(3)]

    def symfill(fn):
        """3x3 symmetric matrix from fn(i, j) evaluated for i <= j."""
        v = [fn(i, j) for (i, j) in SYM6]
        return sym(v)

    R3 = range(3)
    chi, K, Th, al, phi, Pi = u[CHI], u[K_], u[THETA], u[LAPSE], u[PHI], u[PI]
    h = sym(u[H0:H0 + 6])
    A = sym(u[A0:A0 + 6])
    Gh = u[GH0:GH0 + 3]
    beta = u[SHIFT0:SHIFT0 + 3]
    Bv = u[BB0:BB0 + 3]
    dchi, dK, dTh, dal, dphi, dPi = d1[CHI], d1[K_], d1[THETA], d1[LAPSE], d1[PHI], d1[PI]
    dh = [sym([d1[H0 + q][k] for q in range(6)]) for k in R3]        # dh[k][i][j] = d_k h_ij
    dA = [sym([d1[A0 + q][k] for q in range(6)]) for k in R3]
    dGh = [[d1[GH0 + i][k] for k in R3] for i in R3]                  # dGh[i][k] = d_k Gh^i
    dbe = [[d1[SHIFT0 + i][k] for k in R3] for i in R3]               # dbe[i][k] = d_k beta^i
    ddchi, ddal, ddphi = d2[CHI], d2[LAPSE], d2[PHI]
    ddh = [[d2[H0 + PACK[i][j]] for j in R3] for i in R3]             # ddh[i][j][k][l] = d_k d_l h_ij
    ddbe = [d2[SHIFT0 + i] for i in R3]                               # ddbe[i][k][l]

    # ---------------- conformal metric inverse (adjugate over determinant)
    det = (h[0][0] * (h[1][1] * h[2][2] - h[1][2] * h[1][2]) - h[0][1] * (h[0][1] * h[2][2] - h[1][2] * h[0][2])
           + h[0][2] * (h[0][1] * h[1][2] - h[1][1] * h[0][2]))
    idet = 1.0 / det
    adj = {
        (0, 0): h[1][1] * h[2][2] - h[1][2] * h[1][2],
        (0, 1): h[0][2] * h[1][2] - h[0][1] * h[2][2],
        (0, 2): h[0][1] * h[1][2] - h[0][2] * h[1][1],
        (1, 1): h[0][0] * h[2][2] - h[0][2] * h[0][2],
        (1, 2): h[0][1] * h[0][2] - h[0][0] * h[1][2],
        (2, 2): h[0][0] * h[1][1] - h[0][1] * h[0][1],
    }
    hu = symfill(lambda i, j: adj[(i, j)] * idet)
    ichi = 1.0 / chi
    gu = symfill(lambda i, j: chi * hu[i][j])
    gam = symfill(lambda i, j: h[i][j] * ichi)

    # ---------------- Christoffel symbols
    chr1 = [symfill(lambda i, j, k=k: 0.5 * (dh[i][k][j] + dh[j][k][i] - dh[k][i][j])) for k in R3]  # G~_kij
    chr_ = [symfill(lambda i, j, k=k: S(hu[k][l] * chr1[l][i][j] for l in R3)) for k in R3]         # G~^k_ij
    Gt = [S(hu[i][j] * chr_[k][i][j] for i in R3 for j in R3) for k in R3]
    Zt = [0.5 * (Gh[k] - Gt[k]) for k in R3]
    Zl = [S(h[i][k] * Zt[k] for k in R3) for i in R3]
    hud = [S(hu[k][l] * dchi[l] for l in R3) for k in R3]
    half_ichi = 0.5 * ichi
    chrp = [symfill(lambda i, j, k=k: chr_[k][i][j] - half_ichi * (
        (dchi[j] if k == i else zero) + (dchi[i] if k == j else zero) - h[i][j] * hud[k])) for k in R3]

    # ---------------- D_i D_j alpha
    DDa = symfill(lambda i, j: ddal[i][j] - S(chrp[k][i][j] * dal[k] for k in R3))
    D2a = S(gu[i][j] * DDa[i][j] for i in R3 for j in R3)

    # ---------------- d_j Gamma~^k = d_j (h^kn Cn),  Cn = h^lm (d_l h_nm - 1/2 d_n h_lm)
    dhu = [symfill(lambda l, m, j=j: -S(hu[l][a] * hu[m][b] * dh[j][a][b] for a in R3 for b in R3)) for j in R3]
    Cn = [S(hu[l][m] * (dh[l][n][m] - 0.5 * dh[n][l][m]) for l in R3 for m in R3) for n in R3]
    dCn = [[S(dhu[j][l][m] * (dh[l][n][m] - 0.5 * dh[n][l][m]) + hu[l][m] * (ddh[n][m][j][l] - 0.5 * ddh[l][m][j][n])
              for l in R3 for m in R3) for j in R3] for n in R3]  # dCn[n][j] = d_j C_n
    dGt = [[S(dhu[j][k][n] * Cn[n] + hu[k][n] * dCn[n][j] for n in R3) for j in R3] for k in R3]

    # ---------------- Ricci tensors
    # shared pieces: -1/2 h^lm d_l d_m h_ij and the connection-squared terms
    Lap = symfill(lambda i, j: -0.5 * S(hu[l][m] * ddh[i][j][l][m] for l in R3 for m in R3))
    Cu = [[[S(hu[m][l] * chr_[k][l][i] for l in R3) for i in R3] for m in R3] for k in R3]   # Cu[k][m][i] = G~^{k m}_i
    c1u = [[[S(hu[m][l] * chr1[k][l][j] for l in R3) for j in R3] for m in R3] for k in R3]  # c1u[k][m][j] = G~_k^m_j
    T1 = [[S(Cu[k][m][i] * chr1[j][k][m] for k in R3 for m in R3) for j in R3] for i in R3]
    Quad = symfill(lambda i, j: T1[i][j] + T1[j][i] + S(chr_[k][i][m] * c1u[k][m][j] for k in R3 for m in R3))

    def ricci_tilde(G, dG):
        return symfill(lambda i, j: Lap[i][j] + Quad[i][j]
                       + 0.5 * S(h[k][i] * dG[k][j] + h[k][j] * dG[k][i] for k in R3)
                       + 0.5 * S(G[k] * (chr1[i][j][k] + chr1[j][i][k]) for k in R3))

    RtGh = ricci_tilde(Gh, dGh)
    RtGt = ricci_tilde(Gt, dGt)
    DDchi = symfill(lambda i, j: ddchi[i][j] - S(chr_[k][i][j] * dchi[k] for k in R3))
    trDDchi = S(hu[l][m] * DDchi[l][m] for l in R3 for m in R3)
    dchi2 = S(hud[l] * dchi[l] for l in R3)
    quarter_ichi2 = 0.25 * ichi * ichi
    Rchi = symfill(lambda i, j: half_ichi * (DDchi[i][j] + h[i][j] * trDDchi)
                   - quarter_ichi2 * (dchi[i] * dchi[j] + 3.0 * h[i][j] * dchi2))
    Ztdchi = S(Zt[l] * dchi[l] for l in R3)
    Rz = symfill(lambda i, j: RtGh[i][j] + Rchi[i][j] + ichi * (Zl[i] * dchi[j] + Zl[j] * dchi[i] - h[i][j] * Ztdchi))
    Rp = symfill(lambda i, j: RtGt[i][j] + Rchi[i][j])
    Rzs = S(gu[i][j] * Rz[i][j] for i in R3 for j in R3)
    Rs = S(gu[i][j] * Rp[i][j] for i in R3 for j in R3)

    # ---------------- extrinsic curvature
    Aud = [[S(hu[i][k] * A[k][j] for k in R3) for j in R3] for i in R3]   # A~^i_j
    Au = symfill(lambda i, j: S(Aud[i][k] * hu[k][j] for k in R3))         # A~^ij
    A2 = S(A[i][j] * Au[i][j] for i in R3 for j in R3)
    Mi = [S(hu[j][k] * (dA[k][j][i] - S(chr_[l][k][j] * A[l][i] + chr_[l][k][i] * A[j][l] for l in R3))
            for j in R3 for k in R3)
          - 1.5 * ichi * S(Aud[k][i] * dchi[k] for k in R3) - (2.0 / 3.0) * dK[i] for i in R3]
    K3 = K * (1.0 / 3.0)
    Kl = symfill(lambda i, j: (A[i][j] + h[i][j] * K3) * ichi)
    Kud = [[Aud[i][j] + (K3 if i == j else zero) for j in R3] for i in R3]  # K^i_j
    dK3 = [dK[k] * (1.0 / 3.0) for k in R3]
    dKl = [symfill(lambda i, j, k=k: (dA[k][i][j] + dh[k][i][j] * K3 + h[i][j] * dK3[k] - Kl[i][j] * dchi[k]) * ichi)
           for k in R3]
    DK = [symfill(lambda i, j, k=k: dKl[k][i][j] - S(chrp[l][k][i] * Kl[l][j] + chrp[l][k][j] * Kl[i][l] for l in R3))
          for k in R3]                                                      # DK[k][i][j] = D_k K_ij
    Bt = [[[DK[j][i][k] - DK[k][i][j] for k in R3] for j in R3] for i in R3]  # B_ijk

    # Gauss: spatial projection of the 4-Riemann, its "Einstein" combination
    A4 = symfill(lambda i, j: Rp[i][j] + K * Kl[i][j] - S(Kl[i][k] * Kud[k][j] for k in R3))
    A4tr = Rs + (2.0 / 3.0) * K * K - A2
    Gc = symfill(lambda i, j: A4[i][j] - 0.5 * gam[i][j] * A4tr)
    Gcud = [[S(gu[i][a] * Gc[a][j] for a in R3) for j in R3] for i in R3]   # G^i_j
    Gcu = symfill(lambda i, j: S(Gcud[i][b] * gu[b][j] for b in R3))
    Gctr = S(Gcud[i][i] for i in R3)

    # ---------------- scalar field
    dphiu = [S(gu[i][j] * dphi[j] for j in R3) for i in R3]
    dphi2 = S(dphi[i] * dphiu[i] for i in R3)
    g2 = P["g2"]
    X = 0.5 * (Pi * Pi - dphi2)
    FX = 1.0 + 2.0 * g2 * X
    F = X + g2 * X * X
    lam = P["lambda_gb"]
    if general_coupling:
        bphi2 = P["beta"] * phi * phi
        ex = g.exp(-bphi2)
        dlam = P["lambda_lin"] + 0.5 * lam * phi * ex
        ddlam = 0.5 * lam * (1.0 - 2.0 * bphi2) * ex
    else:
        dlam = 0.5 * lam * phi
        ddlam = 0.5 * lam
    DDphi = symfill(lambda i, j: ddphi[i][j] - S(chrp[k][i][j] * dphi[k] for k in R3))
    ial = 1.0 / al
    adphi = ial * S(dal[k] * dphiu[k] for k in R3)                       # a^k d_k phi
    W = symfill(lambda i, j: dlam * (DDphi[i][j] + Kl[i][j] * Pi) + ddlam * dphi[i] * dphi[j])
    Kdphi = [S(Kud[j][i] * dphi[j] for j in R3) for i in R3]             # K_i^j d_j phi
    Vl = [dlam * (dPi[i] + Kdphi[i]) + ddlam * Pi * dphi[i] for i in R3]
    Vu = [S(gu[i][j] * Vl[j] for j in R3) for i in R3]
    Wnn0 = ddlam * Pi * Pi - dlam * adphi

    Bsup = [[[S(gu[s][m] * Bt[m][a][b] for m in R3) for b in R3] for a in R3] for s in R3]
    # B_b^{rs} = g^rm g^sn B_bmn
    Bdup = [[[S(gu[r][m] * S(Bt[b][m][n] * gu[n][s] for n in R3) for m in R3) for s in R3] for r in R3]
            for b in R3]
    B2 = S(Bt[i][j][k] * S(gu[i][a] * Bdup[a][j][k] for a in R3) for i in R3 for j in R3 for k in R3)
    Miu = [S(gu[i][j] * Mi[j] for j in R3) for i in R3]
    M2 = S(Mi[i] * Miu[i] for i in R3)

    # B.V part of H_ij (independent of C and p); only i <= j is used
    E1 = [[S(_eps(e, a, b) * Bsup[q][a][b] for a in R3 for b in R3 if _eps(e, a, b)) for q in R3] for e in R3]
    E2 = [[S(_eps(j, r, q) * Bdup[b][r][q] for r in R3 for q in R3 if _eps(j, r, q)) for j in R3] for b in R3]
    tEJ = [[S(_eps(j, d, q) * E1[e][q] * Vu[d] for d in R3 for q in R3 if _eps(j, d, q))
            + S(_eps(e, c, b) * E2[b][j] * Vl[c] for c in R3 for b in R3 if _eps(e, c, b))
            for j in R3] for e in R3]
    HBV = symfill(lambda i, j: 2.0 * S(gam[i][e] * tEJ[e][j] for e in R3))

    # momentum-constraint source H^0_i and energy density
    Wud = [[S(gu[d][k] * W[k][c] for k in R3) for c in R3] for d in R3]   # W^d_c
    E3 = [[S(_eps(c, a, b) * Bsup[q][a][b] for a in R3 for b in R3 if _eps(c, a, b)) for q in R3] for c in R3]
    H0i = [-4.0 * S(Gcud[c][i] * Vl[c] for c in R3)
           - 2.0 * S(_eps(i, d, q) * E3[c][q] * Wud[d][c] for c in R3 for d in R3 for q in R3 if _eps(i, d, q))
           for i in R3]
    GW = S(Gcu[i][j] * W[i][j] for i in R3 for j in R3)
    rho8 = 0.5 * FX * Pi * Pi - 0.5 * F - 4.0 * GW
    S8i = [-0.5 * FX * Pi * dphi[i] - H0i[i] for i in R3]
    Sig = symfill(lambda i, j: 0.5 * FX * dphi[i] * dphi[j] + 0.5 * gam[i][j] * F)
    Sigtr = 0.5 * FX * dphi2 + 1.5 * F
    # sources as the metric equations see them
    if decoupled:
        rho8m, S8im, Sigm, Sigtrm = zero, [zero] * 3, [[zero] * 3 for _ in R3], zero
    else:
        rho8m, S8im, Sigm, Sigtrm = rho8, S8i, Sig, Sigtr

    # ---------------- per-cell linear system in (C_11..C_33, p)
    Hg = A4tr
    thterm = 0.5 * P["cfac"] * P["k1_2pk2"] * Th + 0.5 * P["k1k2"] * Th
    trace_part = P["b4"] * Hg + 0.5 * P["cfac"] * rho8m + thterm
    KK = symfill(lambda i, j: S(Kl[i][k] * Kud[k][j] for k in R3))
    KmTh = K - 2.0 * Th
    Q = symfill(lambda i, j: Rz[i][j] + KmTh * Kl[i][j] - KK[i][j] - Sigm[i][j]
                + gam[i][j] * (0.5 * Sigtrm - trace_part))
    trW = S(gu[i][j] * W[i][j] for i in R3 for j in R3)
    WG = [[S(W[i][b] * gu[b][a] for b in R3) for a in R3] for i in R3]    # W_i^a

    def bracket(C):
        """gamma_ij (trC trW - tr(CW)) - trC W_ij - trW C_ij + (CW)_ij + (WC)_ij, i<=j."""
        trC = S(gu[i][j] * C[i][j] for i in R3 for j in R3)
        CW = [[S(C[i][a] * WG[j][a] for a in R3) for j in R3] for i in R3]   # C_ia W^a_j (W sym)
        trCW = S(C[i][a] * S(WG[k][a] * gu[k][i] for k in R3) for i in R3 for a in R3)
        return symfill(lambda i, j: gam[i][j] * (trC * trW - trCW) - trC * W[i][j] - trW * C[i][j]
                       + CW[i][j] + CW[j][i])

    def trace_rev(M):
        tr = S(gu[i][j] * M[i][j] for i in R3 for j in R3)
        return symfill(lambda i, j: M[i][j] - 0.5 * gam[i][j] * tr)

    Amat = [[None] * 7 for _ in range(7)]
    one, zero_ = g.const(1.0), g.const(0.0)
    for col, (k, l) in enumerate(SYM6):
        E = [[one if (i, j) in ((k, l), (l, k)) else zero_ for j in R3] for i in R3]
        br = bracket(E)
        Hr = trace_rev(symfill(lambda i, j: -4.0 * br[i][j]))
        for row, (i, j) in enumerate(SYM6):
            Amat[row][col] = E[i][j] if decoupled else E[i][j] - Hr[i][j]
        Amat[6][col] = -8.0 * dlam * (Gcu[k][l] if k == l else 2.0 * Gcu[k][l])
    Gr = trace_rev(Gc)
    for row, (i, j) in enumerate(SYM6):
        Amat[row][6] = zero if decoupled else -4.0 * dlam * Gr[i][j]
    DPi = 1.0 + 3.0 * g2 * Pi * Pi - g2 * dphi2
    Amat[6][6] = DPi
    H0c = trace_rev(symfill(lambda i, j: 4.0 * Gc[i][j] * Wnn0 + HBV[i][j]))
    bvec = [Q[i][j] if decoupled else Q[i][j] + H0c[i][j] for (i, j) in SYM6]
    KDD = S(dphiu[i] * dphiu[j] * (DDphi[i][j] + Kl[i][j] * Pi) for i in R3 for j in R3)
    PiV = S(dphiu[i] * (dPi[i] + Kdphi[i]) for i in R3)
    D2phi = S(gu[i][j] * DDphi[i][j] for i in R3 for j in R3)
    srest = FX * (D2phi + K * Pi + adphi) - 2.0 * g2 * (KDD - 2.0 * Pi * PiV - Pi * Pi * adphi)
    bvec.append(srest + dlam * (8.0 * M2 - 4.0 * B2))

    # Gaussian elimination with partial pivoting; pivots are reported.  Before
    # column kk is eliminated, rows kk+1..6 are compared in turn with row kk,
    # and a row whose entry in column kk is strictly larger in magnitude is
    # exchanged with it (branch-free selects), so that row kk ends with the
    # first largest entry of the column.  In the weak-coupling regime the
    # matrix is identity plus O(lambda', g2) and no exchange is taken.
    M = [row[:] for row in Amat]
    rhs7 = bvec[:]
    pivots = []
    swaps = []  # exchange conditions, for the sign of the determinant
    for kk in range(7):
        for ii in range(kk + 1, 7):
            cnd = g.gtabs(M[ii][kk], M[kk][kk])
            if cnd.op == "c" and cnd.val == 0.0:
                continue
            swaps.append(cnd)
            for jj in range(kk, 7):
                M[kk][jj], M[ii][jj] = g.sel(cnd, M[ii][jj], M[kk][jj]), g.sel(cnd, M[kk][jj], M[ii][jj])
            rhs7[kk], rhs7[ii] = g.sel(cnd, rhs7[ii], rhs7[kk]), g.sel(cnd, rhs7[kk], rhs7[ii])
        piv = M[kk][kk]
        pivots.append(piv)
        ipiv = 1.0 / piv
        for ii in range(kk + 1, 7):
            f = M[ii][kk] * ipiv
            for jj in range(kk + 1, 7):
                M[ii][jj] = M[ii][jj] - f * M[kk][jj]
            rhs7[ii] = rhs7[ii] - f * rhs7[kk]
        M[kk] = [None] * kk + [piv] + [M[kk][jj] * ipiv for jj in range(kk + 1, 7)]
        rhs7[kk] = rhs7[kk] * ipiv
    x = [None] * 7
    for ii in range(6, -1, -1):
        x[ii] = rhs7[ii] - S(M[ii][jj] * x[jj] for jj in range(ii + 1, 7))
    Cs = sym(x[:6])
    ps = x[6]
    # reciprocal pivots and normalised rows, for the near-singularity test
    pivot_check = [1.0 / p_ for p_ in pivots] + [M[kk][jj] for kk in range(7) for jj in range(kk + 1, 7)]

    brs = bracket(Cs)
    Wnn = dlam * ps + Wnn0
    if decoupled:
        S8 = [[zero] * 3 for _ in R3]
    else:
        S8 = symfill(lambda i, j: Sig[i][j] - (4.0 * Gc[i][j] * Wnn - 4.0 * brs[i][j] + HBV[i][j]))
    S8tr = S(gu[i][j] * S8[i][j] for i in R3 for j in R3)

    # ---------------- right-hand sides
    def ad(f):
        return adv[f] if f in adv else zero

    divb = dbe[0][0] + dbe[1][1] + dbe[2][2]
    fb = P["fb"]
    Hcal = Hg - 2.0 * rho8m - 2.0 * P["k1_2pk2"] * Th
    rhs = [None] * NF
    rhs[CHI] = ad(CHI) + (2.0 / 3.0) * chi * (al * K - divb)
    for q, (i, j) in enumerate(SYM6):
        rhs[H0 + q] = (ad(H0 + q) + S(h[k][i] * dbe[k][j] + h[k][j] * dbe[k][i] for k in R3)
                       - (2.0 / 3.0) * h[i][j] * divb - 2.0 * al * A[i][j])
    rhs[K_] = (ad(K_) - D2a + al * (Rzs + K * KmTh) - 3.0 * al * P["k1_1pk2"] * Th
               + 0.5 * al * (S8tr - 3.0 * rho8m) - 0.75 * al * fb * Hcal)
    Xm = symfill(lambda i, j: -DDa[i][j] + al * (Rz[i][j] - S8[i][j]))
    trX = S(hu[k][l] * Xm[k][l] for k in R3 for l in R3)
    for q, (i, j) in enumerate(SYM6):
        AA = S(Aud[k][j] * A[i][k] for k in R3)
        rhs[A0 + q] = (ad(A0 + q) + S(A[k][i] * dbe[k][j] + A[k][j] * dbe[k][i] for k in R3)
                       - (2.0 / 3.0) * A[i][j] * divb + chi * (Xm[i][j] - (1.0 / 3.0) * h[i][j] * trX)
                       + al * (A[i][j] * KmTh - 2.0 * AA))
    Zda = S(Zt[k] * dal[k] for k in R3)
    rhs[THETA] = (ad(THETA) + 0.5 * al * (Rzs - A2 + (2.0 / 3.0) * K * K - 2.0 * Th * K) - chi * Zda
                  - al * P["k1_2pk2"] * Th - al * rho8m - 0.5 * al * fb * Hcal)
    rGam = []
    for i in R3:
        s = ad(GH0 + i) - S(Gt[k] * dbe[i][k] for k in R3) + (2.0 / 3.0) * Gt[i] * divb
        s = s + S(hu[j][k] * ddbe[i][j][k] for j in R3 for k in R3) \
            + (1.0 / 3.0) * S(hu[i][j] * ddbe[k][j][k] for j in R3 for k in R3)
        s = s + 2.0 * P["kappa3"] * ((2.0 / 3.0) * Zt[i] * divb - S(Zt[k] * dbe[i][k] for k in R3))
        t = (S(chr_[i][j][k] * Au[j][k] for j in R3 for k in R3) - 1.5 * ichi * S(Au[i][j] * dchi[j] for j in R3)
             - (2.0 / 3.0) * S(hu[i][j] * dK[j] for j in R3))
        s = s + 2.0 * al * t - 2.0 * S(Au[i][j] * dal[j] for j in R3)
        s = s + 2.0 * S(hu[i][j] * (al * dTh[j] - Th * dal[j] - (2.0 / 3.0) * al * K * Zl[j]) for j in R3)
        s = s - 2.0 * al * P["kappa1"] * Zt[i] - 2.0 * al * S(hu[i][j] * S8im[j] for j in R3)
        AZ = [S(A[j][k] * Zt[k] for k in R3) for j in R3]
        t2 = S(hu[i][j] * (Mi[j] - S8im[j] + dTh[j] - P["kappa1"] * Zl[j] - AZ[j] - K3 * Zl[j]) for j in R3)
        s = s - 2.0 * al * fb * t2
        rGam.append(s)
        rhs[GH0 + i] = s
    rhs[LAPSE] = P["lapse_advec"] * ad(LAPSE) - P["lapse_coeff"] * al * KmTh * P["inv1pa"]
    for i in R3:
        Da = chi * S(hu[i][j] * dal[j] for j in R3)
        rhs[SHIFT0 + i] = P["shift_gamma_coeff"] * Bv[i] - P["a_1pa"] * al * Da
        rhs[BB0 + i] = rGam[i] * P["inv1pa"] - P["eta"] * Bv[i]
        if shift_advec:
            rhs[SHIFT0 + i] = rhs[SHIFT0 + i] + P["shift_advec"] * ad(SHIFT0 + i)
            rhs[BB0 + i] = rhs[BB0 + i] + P["shift_advec"] * (ad(BB0 + i) - ad(GH0 + i) * P["inv1pa"])
    rhs[PHI] = ad(PHI) + al * Pi
    rhs[PI] = ad(PI) + al * ps

    inputs = {n.name: n for n in g.nodes if n.op == "in"}
    # constraint diagnostics: Hamiltonian R + 2/3 K^2 - A_ij A^ij - 2 (8 pi rho)
    # (with the pure Ricci scalar) and momentum M_i - 8 pi S_i
    # in the decoupling limit the metric constraints carry no scalar sources
    constraints = [Hg - 2.0 * rho8m] + [Mi[i] - S8im[i] for i in R3]
    return dict(graph=g, rhs=rhs, pivots=pivots, pivot_check=pivot_check, swaps=swaps, inputs=inputs, params=P,
                theta=[P["lambda_gb"], P["g2"]], solution=x, constraints=constraints,
                scalar_parts=dict(X=X, Pi=Pi, GW=GW, g2=g2, Gcu=Gcu, Cs=Cs, M2=M2, B2=B2, dlam=dlam))


def coupling(b):
    """Gauss-Bonnet invariant with the solved C_ij (the scalar row's reading:
    8 G^kl C_kl + 8 M_i M^i - 4 B_ijk B^ijk), the weak-coupling indicators
    |lambda'(phi)| sqrt|L_GB| and |2 g2 X|, and the determinant of the
    per-cell system, added to the graph on request."""
    q = b["scalar_parts"]
    g = q["X"].g
    Gcu, Cs = q["Gcu"], q["Cs"]
    gc = g.sum(Gcu[i][j] * Cs[i][j] for i in range(3) for j in range(3))
    lgb = 8.0 * gc + 8.0 * q["M2"] - 4.0 * q["B2"]
    det = b["pivots"][0]
    for pv in b["pivots"][1:]:
        det = det * pv
    for cnd in b["swaps"]:  # each exchange taken flips the sign
        det = g.sel(cnd, -det, det)
    return [lgb, g.fabs(q["dlam"]) * g.sqrt(g.fabs(lgb)), g.fabs(2.0 * q["g2"] * q["X"]), det]


def energies(b):
    """Energy densities n^a n^b T_ab of the canonical, X^2 and Gauss-Bonnet
    terms (the three pieces of rho8, divided by 8 pi), added to the graph of
    build() on request only, so that the other outputs keep their node order."""
    q = b["scalar_parts"]
    X, Pi, GW, g2 = q["X"], q["Pi"], q["GW"], q["g2"]
    inv8pi = 1.0 / (8.0 * math.pi)
    return [(0.5 * Pi * Pi - 0.5 * X) * inv8pi,
            g2 * (X * Pi * Pi - 0.5 * X * X) * inv8pi,
            (-4.0 * GW) * inv8pi]
