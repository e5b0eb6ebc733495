"""Independent covariant reference for the pointwise 3+1 right-hand side.

Test infrastructure.  A random smooth spacetime (lapse, shift, 3-metric, scalar
phi, Z4 vector Z^mu, all quadratic polynomials in (t, x, y, z)) is built at the
origin.  Its free second time derivatives (d_t^2 gamma_ij, d_t^2 phi) and the
time derivatives d_t Z^mu are solved for so that the covariant field equations
hold at the origin:

  * modified Z4 (trace reversal with hat g^{mu nu} = g^{mu nu} - b n^mu n^nu):
      G^{mu nu} + hat g^{nu b} nabla_b Z^mu + hat g^{mu b} nabla_b Z^nu
        - hat g^{mu nu} nabla_a Z^a - kappa1 (n^mu Z^nu + n^nu Z^mu
        + kappa2 g^{mu nu} n_a Z^a) = 8 pi T^{mu nu}
  * 4dST stress: 8 pi T^mu_nu = 1/2 F_X d^mu phi d_nu phi + 1/2 delta^mu_nu F
        - delta^{mu g a b}_{nu d r s} R^{r s}_{a b} nabla^d nabla_g lambda(phi)
  * scalar: nabla_mu (F_X nabla^mu phi) + lambda'(phi) L_GB = 0
  with X = -1/2 (d phi)^2, F_X = 1 + 2 g2 X, F = X + g2 X^2,
  lambda = lambda_gb phi^2 / 4, L_GB = Riem^2 - 4 Ric^2 + R^2.

Everything is computed by automatic differentiation of the 4-metric (torch,
float64), with no 3+1 formula in sight.  The conformal 3+1 variables of that
spacetime and their exact spatial derivatives are then handed to the oracle's
pointwise function, whose output must equal the true time derivatives.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch
from torch.func import jacfwd

torch.set_default_dtype(torch.float64)


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


_EPS4 = torch.zeros(4, 4, 4, 4)
for _p in itertools.permutations(range(4)):
    _EPS4[_p] = _perm_sign(_p)
# generalised Kronecker delta: product of two permutation symbols
DELTA4 = torch.einsum("abcd,efgh->abcdefgh", _EPS4, _EPS4)

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def det3(m):
    return (m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
            - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
            + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))


def inv3(m):
    d = det3(m)
    c = torch.stack([
        torch.stack([m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1], m[0, 2] * m[2, 1] - m[0, 1] * m[2, 2],
                     m[0, 1] * m[1, 2] - m[0, 2] * m[1, 1]]),
        torch.stack([m[1, 2] * m[2, 0] - m[1, 0] * m[2, 2], m[0, 0] * m[2, 2] - m[0, 2] * m[2, 0],
                     m[0, 2] * m[1, 0] - m[0, 0] * m[1, 2]]),
        torch.stack([m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0], m[0, 1] * m[2, 0] - m[0, 0] * m[2, 1],
                     m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0]]),
    ])
    return c / d


class Poly:
    """Quadratic polynomial field c0 + c1.x + 1/2 x.c2.x (x = (t,x,y,z)), any leading shape."""

    def __init__(self, c0, c1, c2):
        self.c0, self.c1, self.c2 = c0, c1, c2

    def __call__(self, x):
        return self.c0 + self.c1 @ x + 0.5 * torch.einsum("...ab,a,b->...", self.c2, x, x)


def _sym4(a):
    return 0.5 * (a + a.transpose(-1, -2))


class RandomSpacetime:
    def __init__(self, seed, scale=0.15):
        g = np.random.default_rng(seed)

        def r(*s):
            return torch.tensor(g.uniform(-1, 1, size=s))

        s = scale
        self.alpha = Poly(1.1 + 0.1 * r(), s * r(4), _sym4(s * r(4, 4)))
        self.beta = Poly(s * r(3), s * r(3, 4), _sym4(s * r(3, 4, 4)))
        g0 = torch.eye(3) + s * _sym4(r(3, 3))
        g1 = s * r(3, 3, 4)
        g1 = 0.5 * (g1 + g1.transpose(0, 1))
        g2 = _sym4(s * r(3, 3, 4, 4))
        g2 = 0.5 * (g2 + g2.transpose(0, 1))
        self.gam = Poly(g0, g1, g2)
        self.phi = Poly(0.5 + 0.1 * r(), 0.3 * r(4), _sym4(0.3 * r(4, 4)))
        self.Z = Poly(s * r(4), s * r(4, 4), torch.zeros(4, 4, 4))
        self.B = Poly(s * r(3), s * r(3, 4), torch.zeros(3, 4, 4))

    # unknowns: d_t^2 gamma_ij (6), d_t Z^mu (4), d_t^2 phi (1)
    def set_unknowns(self, xi):
        g2 = self.gam.c2.clone()
        for q, (i, j) in enumerate(SYM):
            g2[i, j, 0, 0] = xi[q]
            g2[j, i, 0, 0] = xi[q]
        self.gam = Poly(self.gam.c0, self.gam.c1, g2)
        z1 = self.Z.c1.clone()
        z1[:, 0] = xi[6:10]
        self.Z = Poly(self.Z.c0, z1, self.Z.c2)
        p2 = self.phi.c2.clone()
        p2[0, 0] = xi[10]
        self.phi = Poly(self.phi.c0, self.phi.c1, p2)

    # ---- 4-geometry
    def metric(self, x):
        a = self.alpha(x)
        b = self.beta(x)
        gm = self.gam(x)
        bl = gm @ b
        g00 = -a * a + bl @ b
        top = torch.cat([g00.reshape(1), bl])
        rest = torch.cat([bl.reshape(3, 1), gm], dim=1)
        return torch.cat([top.reshape(1, 4), rest], dim=0)

    def metric_inv(self, x):
        a = self.alpha(x)
        b = self.beta(x)
        gi = inv3(self.gam(x))
        a2 = a * a
        top = torch.cat([(-1.0 / a2).reshape(1), b / a2])
        rest = torch.cat([(b / a2).reshape(3, 1), gi - torch.outer(b, b) / a2], dim=1)
        return torch.cat([top.reshape(1, 4), rest], dim=0)

    def christoffel(self, x):
        """Gam^l_{mn} = 1/2 g^{ls} (d_m g_{sn} + d_n g_{sm} - d_s g_{mn})."""
        gi = self.metric_inv(x)
        dg = jacfwd(self.metric)(x)  # [m, n, l] = d_l g_mn
        dm_gsn = torch.einsum("snm->smn", dg)
        dn_gsm = dg
        ds_gmn = torch.einsum("mns->smn", dg)
        return 0.5 * torch.einsum("ls,smn->lmn", gi, dm_gsn + dn_gsm - ds_gmn)

    def geometry(self, x):
        g = self.metric(x)
        gi = self.metric_inv(x)
        Gam = self.christoffel(x)
        dGam = jacfwd(self.christoffel)(x)  # [r, n, s, m] = d_m Gam^r_{ns}
        Riem = (torch.einsum("rnsm->rsmn", dGam) - torch.einsum("rmsn->rsmn", dGam)
                + torch.einsum("rml,lns->rsmn", Gam, Gam) - torch.einsum("rnl,lms->rsmn", Gam, Gam))
        return g, gi, Gam, Riem


def field_equations(st: RandomSpacetime, params: dict, x0=None):
    """Residuals of the modified Z4 equations (10, upper indices mu<=nu) and the
    scalar equation at x0, plus the geometric objects used."""
    if x0 is None:
        x0 = torch.zeros(4)
    lam_gb, g2c = params["lambda_gb"], params["g2"]
    b, k1, k2 = params["b_gauge"], params["kappa1"], params["kappa2"]
    g, gi, Gam, Riem = st.geometry(x0)
    Ric = torch.einsum("rsrn->sn", Riem)
    Rs = torch.einsum("sn,sn->", gi, Ric)
    G_low = Ric - 0.5 * g * Rs
    G_up = gi @ G_low @ gi

    phi = st.phi(x0)
    dphi = jacfwd(st.phi)(x0)
    ddphi = jacfwd(jacfwd(st.phi))(x0)
    beta = params.get("beta", 0.0)
    ex = torch.exp(-beta * phi * phi)
    dlam = params.get("lambda_lin", 0.0) + 0.5 * lam_gb * phi * ex
    ddlam = 0.5 * lam_gb * (1.0 - 2.0 * beta * phi * phi) * ex
    dl = dlam * dphi
    ddl = ddlam * torch.outer(dphi, dphi) + dlam * ddphi
    nnl = ddl - torch.einsum("rmn,r->mn", Gam, dl)  # nabla_m nabla_n lambda
    Rud = torch.einsum("sk,rkab->rsab", gi, Riem)   # R^{rs}_{ab}
    Dl = gi @ nnl                                   # nabla^d nabla_g lambda  [d, g]
    P = torch.einsum("mgabndrs,rsab,dg->mn", DELTA4, Rud, Dl)

    def Xf(x):
        gi_ = st.metric_inv(x)
        dp = jacfwd(st.phi)(x)
        return -0.5 * dp @ gi_ @ dp

    X = Xf(x0)
    dX = jacfwd(Xf)(x0)
    FX = 1.0 + 2.0 * g2c * X
    F = X + g2c * X * X
    dphi_up = gi @ dphi
    T8_mixed = 0.5 * FX * torch.outer(dphi_up, dphi) + 0.5 * torch.eye(4) * F - P  # [mu, nu] = T^mu_nu
    T8_up = T8_mixed @ gi

    a = st.alpha(x0)
    bvec = st.beta(x0)
    n_up = torch.cat([(1.0 / a).reshape(1), -bvec / a])
    n_low = torch.tensor([-1.0, 0.0, 0.0, 0.0]) * a
    ghat = gi - b * torch.outer(n_up, n_up)
    Z = st.Z(x0)
    dZ = jacfwd(st.Z)(x0)  # [a, b] = d_b Z^a
    nZ = dZ + torch.einsum("abl,l->ab", Gam, Z)  # nabla_b Z^a
    div = torch.trace(nZ)
    nZdot = n_low @ Z
    # hat g^{nu b} nabla_b Z^mu = (nZ @ ghat)[mu, nu]
    # decoupling limit: the scalar is a test field, the metric equations are vacuum
    source = 0.0 * T8_up if params.get("decoupled", 0.0) else T8_up
    E = (G_up + nZ @ ghat + (nZ @ ghat).T - ghat * div
         - k1 * (torch.outer(n_up, Z) + torch.outer(Z, n_up) + k2 * gi * nZdot) - source)

    box = torch.einsum("mn,mn->", gi, ddphi - torch.einsum("rmn,r->mn", Gam, dphi))
    R_low = torch.einsum("rk,ksmn->rsmn", g, Riem)
    R_up = torch.einsum("sa,mb,nc,rabc->rsmn", gi, gi, gi, Riem)
    Kret = torch.einsum("rsmn,rsmn->", R_low, R_up)
    Ric_up = gi @ Ric @ gi
    LGB = Kret - 4.0 * torch.einsum("mn,mn->", Ric, Ric_up) + Rs * Rs
    Ephi = FX * box + dphi_up @ (2.0 * g2c * dX) + dlam * LGB

    res = torch.stack([E[m, n] for m in range(4) for n in range(m, 4)] + [Ephi])
    # n^mu n^nu T_mu nu (times 8 pi) of each term of the action: canonical X,
    # g2 X^2 and the Gauss-Bonnet coupling
    T_parts = [0.5 * torch.outer(dphi_up, dphi) + 0.5 * torch.eye(4) * X,
               g2c * X * torch.outer(dphi_up, dphi) + 0.5 * torch.eye(4) * g2c * X * X,
               -P]
    rho8 = torch.stack([n_low @ (Tm @ gi) @ n_low for Tm in T_parts])
    return res, dict(g=g, gi=gi, Riem=Riem, R_low=R_low, n_up=n_up, LGB=LGB, rho8=rho8)


def solve_unknowns(st: RandomSpacetime, params: dict):
    """The field equations are affine in the 11 unknowns; solve them exactly."""
    xi0 = torch.zeros(11)
    st.set_unknowns(xi0)
    r0, _ = field_equations(st, params)
    J = torch.zeros(11, 11)
    for k in range(11):
        e = torch.zeros(11)
        e[k] = 1.0
        st.set_unknowns(e)
        rk, _ = field_equations(st, params)
        J[:, k] = rk - r0
    xi = torch.linalg.solve(J, -r0)
    st.set_unknowns(xi)
    r, info = field_equations(st, params)
    return xi, r, info


def conformal_variables(st: RandomSpacetime):
    """Function x -> the 27 evolved variables of the spacetime at x."""

    def gam(x):
        return st.gam(x)

    def gam_conf(x):
        gm = st.gam(x)
        chi = det3(gm) ** (-1.0 / 3.0)
        return chi * gm

    def shift_low(x):
        return st.gam(x) @ st.beta(x)

    def U(x):
        a = st.alpha(x)
        b = st.beta(x)
        gm = gam(x)
        gi = inv3(gm)
        dg = jacfwd(gam)(x)  # [i, j, mu]
        dgs = dg[:, :, 1:]   # [i, j, k] = d_k g_ij
        # 3-Christoffel Gam^k_ij = 1/2 g^kl (d_i g_lj + d_j g_li - d_l g_ij)
        c1 = torch.einsum("lji->lij", dgs)
        c2 = dgs
        c3 = torch.einsum("ijl->lij", dgs)
        chr3 = 0.5 * torch.einsum("kl,lij->kij", gi, c1 + c2 - c3)
        bl = shift_low(x)
        dbl = jacfwd(shift_low)(x)[:, 1:]   # [j, i] = d_i beta_j
        Db = dbl.T - torch.einsum("kij,k->ij", chr3, bl)  # D_i beta_j [i, j]
        Kij = -(dg[:, :, 0] - Db - Db.T) / (2.0 * a)
        chi = det3(gm) ** (-1.0 / 3.0)
        h = chi * gm
        trK = torch.einsum("ij,ij->", gi, Kij)
        At = chi * (Kij - gm * trK / 3.0)
        Z = st.Z(x)
        Theta = a * Z[0]
        Zl = bl * Z[0] + gm @ Z[1:]
        hi = gi / chi
        dh = jacfwd(gam_conf)(x)[:, :, 1:]  # [i, j, k] = d_k h_ij
        c1 = torch.einsum("lji->lij", dh)
        c2 = dh
        c3 = torch.einsum("ijl->lij", dh)
        chrc = 0.5 * torch.einsum("kl,lij->kij", hi, c1 + c2 - c3)
        Gt = torch.einsum("jk,ijk->i", hi, chrc)
        Gh = Gt + 2.0 * hi @ Zl
        dphi = jacfwd(st.phi)(x)
        Pi = (dphi[0] - b @ dphi[1:]) / a
        Bv = st.B(x)
        parts = [chi.reshape(1), torch.stack([h[i, j] for i, j in SYM]), trK.reshape(1),
                 torch.stack([At[i, j] for i, j in SYM]), Theta.reshape(1), Gh, a.reshape(1), b, Bv,
                 st.phi(x).reshape(1), Pi.reshape(1)]
        return torch.cat(parts)

    return U


def reference_point(seed, params):
    """Solve a random spacetime and return (u, d1, d2, dt_true, extra) at the origin."""
    st = RandomSpacetime(seed)
    xi, res, info = solve_unknowns(st, params)
    U = conformal_variables(st)
    x0 = torch.zeros(4)
    u = U(x0)
    J = jacfwd(U)(x0)
    H = jacfwd(jacfwd(U))(x0)
    d1 = J[:, 1:]
    d2 = torch.stack([H[:, 1 + i, 1 + j] for i, j in SYM], dim=1)
    dt_true = J[:, 0]
    # C_ij = R_{i mu j nu} n^mu n^nu and p = n^mu d_mu Pi
    n_up = info["n_up"]
    R_low = info["R_low"]
    C = torch.einsum("imjn,m,n->ij", R_low[1:, :, 1:, :], n_up, n_up)

    def Pi_f(x):
        return U(x)[26]

    p_true = n_up @ jacfwd(Pi_f)(x0)
    return dict(u=u.numpy(), d1=d1.numpy(), d2=d2.numpy(), dt=dt_true.numpy(),
                C=np.array([C[i, j].item() for i, j in SYM]), p=p_true.item(),
                residual=res.abs().max().item(), LGB=info["LGB"].item(), rho8=info["rho8"].numpy())
