"""CPU checks of the generated pointwise code (host build of gen_rhs.inc and
gen_vjp.inc): the forward right-hand side against the oracle's pointwise
right-hand side on random inputs, and the reverse-mode code against central
differences of the forward code."""
import numpy as np
import pytest

import hostgen as H
from oracle import oracle as O
from parity_util import exchange_state as _exchange_state, no_exchange_pivots as _no_exchange_pivots
from paper_2309_06225_amd import inputs as I
from paper_2309_06225_amd.codegen.ccz4_4dst import merged_adv

NF = 27


def _point(rng):
    """Random pointwise inputs near a perturbed puncture background."""
    u = 0.05 * rng.standard_normal(NF)
    u[I.IDX["chi"]] = 0.6 + 0.3 * rng.random()
    for n in ("h11", "h22", "h33"):
        u[I.IDX[n]] += 1.0
    u[I.IDX["lapse"]] = 0.5 + 0.4 * rng.random()
    d1 = 0.2 * rng.standard_normal((NF, 3))
    d2 = 0.2 * rng.standard_normal((NF, 6))
    adv = 0.2 * rng.standard_normal((NF, 3))
    return u, d1, d2, adv


def _record(u, d1, d2, adv, sa):
    """The derivative-record vector the generated code reads: advection sums
    beta^k adv_k for the advected fields (shift and B only with shift
    advection); the Kreiss-Oliger slots stay zero (the stage adds them)."""
    beta = u[I.IDX["shift1"]:I.IDX["shift3"] + 1]
    advsum = np.array([np.dot(beta, adv[f]) for f in range(NF)])
    if not sa:
        advsum[19:25] = 0.0
    return H.pack_inputs(d1, d2, advsum)


@pytest.mark.parametrize("sa", [0, 1])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_generated_rhs_matches_oracle_point(sa, seed):
    rng = np.random.default_rng(seed)
    p = I.default_params(shift_advec=float(sa), lambda_gb=0.3, g2=0.05, lambda_lin=0.15, beta=1.5)
    u, d1, d2, adv = _point(rng)
    if not sa:
        adv[19:25] = 0.0  # the oracle multiplies them by shift_advec = 0 anyway
    o, _, flags = O.rhs_point(I.params_vector(p), u, d1, d2, adv)
    D = _record(u, d1, d2, adv, sa)
    g, bad = H.rhs_point(H.point_params(p), u, D, sa)
    assert bad == 0 and flags == 0
    # advection sums that the stencil stage carries in the Kreiss-Oliger slot
    for f in merged_adv(bool(sa)):
        g[f] += D[144 + f]
    np.testing.assert_allclose(g, o, rtol=1e-12, atol=1e-12 * np.abs(o).max())


@pytest.mark.parametrize("sa", [0, 1])
def test_generated_vjp_matches_central_differences(sa):
    # the reverse code is that of the quadratic coupling (the adjoint refuses
    # the linear and exponential terms)
    rng = np.random.default_rng(7 + sa)
    p = I.default_params(shift_advec=float(sa), lambda_gb=0.3, g2=0.05)
    pp = H.point_params(p)
    u, d1, d2, adv = _point(rng)
    D = _record(u, d1, d2, adv, sa)
    w = rng.standard_normal(NF)
    ub, Db, tb = H.vjp_point(pp, u, D, w, sa)
    du = rng.standard_normal(NF)
    dD = rng.standard_normal(D.shape)
    dD[171:] = 0.0  # Kreiss-Oliger slots are not read by the pointwise code
    if not sa:
        dD[144 + 19:144 + 25] = 0.0
    dth = np.array([0.7, -0.4])
    h = 1e-6

    def J(s):
        q = pp.copy()
        q[0] += s * dth[0]
        q[1] += s * dth[1]
        r, _ = H.rhs_point(q, u + s * du, D + s * dD, sa)
        return float(w @ r)

    fd = (J(h) - J(-h)) / (2 * h)
    ad = float(ub @ du + Db @ dD + tb @ dth)
    assert ad == pytest.approx(fd, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("sa", [0, 1])
def test_generated_solve_exchanges_rows(sa):
    """The per-cell system is solved with partial pivoting: at a state whose
    system has a vanishing first diagonal entry but a condition number of
    order one, the generated code (host build) matches the oracle's
    right-hand side and raises no near-singularity flag, where elimination
    without row exchanges meets a zero pivot."""
    u, d1, d2, lg = _exchange_state()
    p = I.default_params(shift_advec=float(sa), lambda_gb=lg, g2=0.1)
    adv = np.zeros((NF, 3))
    o, ex, flags = O.rhs_point(I.params_vector(p), u, d1, d2, adv)
    A = ex["A"]
    assert np.linalg.cond(A) < 10.0
    assert abs(_no_exchange_pivots(A)[0]) < 1e-14 * np.abs(A).max()
    assert flags == 0
    D = _record(u, d1, d2, adv, sa)
    g, bad = H.rhs_point(H.point_params(p), u, D, sa)
    assert bad == 0
    for f in merged_adv(bool(sa)):
        g[f] += D[144 + f]
    np.testing.assert_allclose(g, o, rtol=1e-11, atol=1e-11 * np.abs(o).max())


def test_generated_vjp_through_row_exchanges():
    """The reverse code differentiates through the exchanges the solve takes:
    at the state of test_generated_solve_exchanges_rows (the same exchanges
    are taken at every point of the difference stencil), it matches central
    differences of the forward code."""
    u, d1, d2, lg = _exchange_state()
    p = I.default_params(lambda_gb=lg, g2=0.1)
    pp = H.point_params(p)
    adv = np.zeros((NF, 3))
    D = _record(u, d1, d2, adv, 0)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(NF)
    ub, Db, tb = H.vjp_point(pp, u, D, w, 0)
    du = rng.standard_normal(NF)
    dD = rng.standard_normal(D.shape)
    dD[171:] = 0.0
    dD[144 + 19:144 + 25] = 0.0
    dth = np.array([0.7, -0.4])
    h = 1e-6

    def J(s):
        q = pp.copy()
        q[0] += s * dth[0]
        q[1] += s * dth[1]
        r, bad = H.rhs_point(q, u + s * du, D + s * dD, 0)
        assert bad == 0
        return float(w @ r)

    fd = (J(h) - J(-h)) / (2 * h)
    ad = float(ub @ du + Db @ dD + tb @ dth)
    assert ad == pytest.approx(fd, rel=1e-6, abs=1e-8)
