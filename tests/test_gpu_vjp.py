"""GPU vector-Jacobian products against the CPU oracle's complex-step tangents
and against central finite differences."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2309_06225_amd import adjoint as A
from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I
from parity_util import exchange_state, no_exchange_pivots, quadratic_box

DEV = "cuda"
H_CS = 1e-30


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    G.lib()


def _state(dims, dx, seed, amp=0.02):
    u = I.puncture(dims, dx, centre=(0.7, -0.4, 0.3), phi_fn=I.shell_pulse(0.2, 1.5))
    rng = np.random.default_rng(seed)
    u += amp * rng.standard_normal(u.shape) * (np.abs(u) + 0.1)
    u[I.IDX["lapse"]] = np.abs(u[I.IDX["lapse"]]) + 0.2
    u[I.IDX["chi"]] = np.abs(u[I.IDX["chi"]]) + 0.1
    return u


def _interior_mask(shape):
    m = np.zeros(shape, bool)
    m[:, 3:-3, 3:-3, 3:-3] = True
    return m


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 1), (5, 1, 4), (70, 2, 2)])
def test_rhs_vjp_degenerate_boxes(dims):
    """The reverse on boxes of a single cell, one or two cells thick, or with
    a row longer than a wave: <w, J v + J_theta dth> from the oracle's
    complex-step tangent equals <VJP(w), (v, dth)> (frozen ghosts, so the
    transposed stencils reach into the ghost layers from every side)."""
    print("case: RHS VJP degenerate box", dims, flush=True)
    p = I.default_params(shift_advec=1.0, lambda_gb=0.3, g2=0.05)
    dx = 0.4
    u = _state(dims, dx, 4)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(u.shape)
    dth = np.array([0.7, -0.4])
    w = rng.standard_normal(u.shape) * _interior_mask(u.shape)
    _, jim = O.rhs_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx)
    lhs = np.sum(w * jim / H_CS * _interior_mask(u.shape))
    ut = torch.from_numpy(u).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    ubar = torch.zeros_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    box = G.box_of(ut, dx)
    ws = G.alloc_workspace(G.vjp_workspace_bytes(box))
    G.rhs_vjp(G.make_params(p), box, ut, wt, ubar, tbar, ws)
    rhs = float(np.sum(ubar.cpu().numpy() * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)


def test_rhs_vjp_through_row_exchanges():
    """The reverse of the pivoting solve on the GPU: on the 9^3 quadratic box
    whose central cell's per-cell system has a vanishing first diagonal entry
    (so the solve exchanges rows there), <w, J v + J_theta dth> from the
    oracle's complex-step tangent equals <VJP(w), (v, dth)>."""
    print("case: RHS VJP 9^3 quadratic box, per-cell system with a zero first pivot", flush=True)
    u0, d1, d2, lg = exchange_state()
    p = I.default_params(lambda_gb=lg, g2=0.1)
    _, ex, _ = O.rhs_point(I.params_vector(p), u0, d1, d2, d1)
    assert abs(no_exchange_pivots(ex["A"])[0]) < 1e-14
    dims, dx = (9, 9, 9), 0.05
    u = quadratic_box(u0, d1, d2, dims, dx)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(u.shape)
    dth = np.array([0.7, -0.4])
    w = rng.standard_normal(u.shape) * _interior_mask(u.shape)
    _, jim = O.rhs_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx)
    lhs = np.sum(w * jim / H_CS * _interior_mask(u.shape))
    ut = torch.from_numpy(u).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    ubar = torch.zeros_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    box = G.box_of(ut, dx)
    ws = G.alloc_workspace(G.vjp_workspace_bytes(box))
    G.rhs_vjp(G.make_params(p), box, ut, wt, ubar, tbar, ws)
    rhs = float(np.sum(ubar.cpu().numpy() * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)


@pytest.mark.parametrize("fd_order", [4.0, 6.0])
@pytest.mark.parametrize("shift_advec", [0.0, 1.0])
def test_rhs_vjp_dot_product_vs_oracle_tangent(shift_advec, fd_order):
    print("case: RHS VJP 11x9x7 shift_advec", shift_advec, "fd_order", fd_order, flush=True)
    p = I.default_params(shift_advec=shift_advec, lambda_gb=0.3, g2=0.05, fd_order=fd_order)
    dims, dx = (11, 9, 7), 0.4
    u = _state(dims, dx, 1)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(u.shape)
    dth = np.array([0.7, -0.4])
    w = rng.standard_normal(u.shape) * _interior_mask(u.shape)
    # oracle tangent J v + J_theta dth by complex step
    _, jim = O.rhs_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx)
    lhs = np.sum(w * jim / H_CS * _interior_mask(u.shape))
    ut = torch.from_numpy(u).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    ubar = torch.zeros_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    box = G.box_of(ut, dx)
    ws = G.alloc_workspace(G.vjp_workspace_bytes(box))
    G.rhs_vjp(G.make_params(p), box, ut, wt, ubar, tbar, ws)
    rhs = float(np.sum(ubar.cpu().numpy() * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)
    # accumulation: a second call adds the same amount again
    ub1, tb1 = ubar.clone(), tbar.clone()
    G.rhs_vjp(G.make_params(p), box, ut, wt, ubar, tbar, ws)
    assert torch.allclose(ubar, 2 * ub1, rtol=1e-14, atol=0)
    assert torch.allclose(tbar, 2 * tb1, rtol=1e-14, atol=0)
    # determinism
    ub2 = torch.zeros_like(ut)
    tb2 = torch.zeros(2, dtype=torch.float64, device=DEV)
    G.rhs_vjp(G.make_params(p), box, ut, wt, ub2, tb2, ws)
    assert torch.equal(ub2, ub1) and torch.equal(tb2, tb1)
    # another stencil variant gives the same bits
    ub3 = torch.zeros_like(ut)
    tb3 = torch.zeros(2, dtype=torch.float64, device=DEV)
    v0 = G.get_tile_variant()
    G.set_tile_variant(6 if v0 != 6 else 0)
    try:
        G.rhs_vjp(G.make_params(p), box, ut, wt, ub3, tb3, ws)
    finally:
        G.set_tile_variant(v0)
    assert torch.equal(ub3, ub1) and torch.equal(tb3, tb1)


def test_rhs_vjp_reaches_ghosts():
    """Cotangents flow into ghost cells (they are inputs of the stencils)."""
    p = I.default_params()
    u = _state((8, 8, 8), 0.5, 3)
    w = np.zeros_like(u)
    w[:, 3, 3, 3] = 1.0  # first interior cell
    ut, wt = torch.from_numpy(u).to(DEV), torch.from_numpy(w).to(DEV)
    ubar = torch.zeros_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    box = G.box_of(ut, 0.5)
    G.rhs_vjp(G.make_params(p), box, ut, wt, ubar, tbar, G.alloc_workspace(G.vjp_workspace_bytes(box)))
    ub = ubar.cpu().numpy()
    assert np.abs(ub[:, 0:3, 3, 3]).max() > 0  # z-ghosts below the cell
    assert np.abs(ub[:, 3, 3, 7:]).max() == 0   # beyond the stencil reach


@pytest.mark.parametrize("fd_order", [4.0, 6.0])
def test_rk4_step_vjp_vs_oracle_tangent(fd_order):
    print("case: RK4 step VJP 10x8x9 fd_order", fd_order, flush=True)
    p = I.default_params(lambda_gb=0.3, g2=0.05, shift_advec=1.0 if fd_order == 6.0 else 0.0, fd_order=fd_order)
    dims, dx, dt = (10, 8, 9), 0.4, 0.1
    u = _state(dims, dx, 5, amp=0.01)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(u.shape)
    dth = np.array([-0.3, 0.9])
    w = rng.standard_normal(u.shape)
    _, uim = O.rk4_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx, dt, 1, periodic=False)
    lhs = np.sum(w * uim / H_CS)
    ut = torch.from_numpy(u).to(DEV)
    traj = A.Trajectory(p, G.box_of(ut, dx), dt, 1)
    P = traj._params([p["lambda_gb"], p["g2"]])
    bufs = [ut.clone() for _ in range(4)]
    traj.step(P, ut, traj._accbuf(ut.device), bufs)
    u2, u3, u4 = bufs[:3]
    ubar = torch.empty_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    ws = G.alloc_workspace(G.step_vjp_workspace_bytes(traj.box))
    G.rk4_step_vjp(P, traj.box, dt, ut, u2, u3, u4, torch.from_numpy(w).to(DEV), ubar, tbar, ws)
    rhs = float(np.sum(ubar.cpu().numpy() * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)


def _cfg3(n=64, dx=0.25):
    return I.single_puncture(n, dx)


def _grad_and_fd(n, dx, nsteps, every, r_in, r_out, eps_list, seed=0):
    p = I.default_params()
    dt = 0.25 * dx
    u0 = _cfg3(n, dx)
    mask = torch.from_numpy(I.shell_mask((n, n, n), dx, r_in, r_out)).to(DEV)
    ut = torch.from_numpy(u0).to(DEV)
    traj = A.Trajectory(p, G.box_of(ut, dx), dt, nsteps, every=every)
    theta = torch.tensor([p["lambda_gb"], p["g2"]], dtype=torch.float64, requires_grad=True)
    u0t = ut.clone().requires_grad_(True)
    J = A.shell_phi2(A.Evolve.apply(theta, u0t, traj), mask)
    J.backward()
    gth = theta.grad.numpy().copy()
    gu = u0t.grad.cpu().numpy()

    def Jof(th, uinit):
        with torch.no_grad():
            un, _ = traj.forward(th, uinit)
            return float(A.shell_phi2(un, mask))

    th0 = [p["lambda_gb"], p["g2"]]
    rng = np.random.default_rng(seed)
    v = np.zeros_like(u0)
    v[I.IDX["phi"]] = rng.standard_normal(u0.shape[1:])
    vt = torch.from_numpy(v).to(DEV)
    fds = {}
    for eps in eps_list:
        fd_th = []
        for q in range(2):
            tp, tm = list(th0), list(th0)
            tp[q] += eps
            tm[q] -= eps
            fd_th.append((Jof(tp, ut) - Jof(tm, ut)) / (2 * eps))
        fd_u = (Jof(th0, ut + eps * vt) - Jof(th0, ut - eps * vt)) / (2 * eps)
        fds[eps] = (np.array(fd_th), fd_u)
    return float(J.detach()), gth, float(np.sum(gu * v)), fds


def test_trajectory_gradient_vs_central_fd_cfg3():
    """64^3 puncture + scalar, dx = M/4, 50 RK4 steps, checkpoints every 10;
    J = sum over 8 < r < 10 of phi^2, d J / d(lambda_gb, g2) and d J / d phi_0 . v
    against central differences.  With step 1e-6 the difference quotient of
    the couplings is limited by the rounding of J itself: its floor is
    ulp(J) / (2 h |J'|) (about 1.2e-6 here, J ~ 0.045, J' ~ 3e-6), so the
    tolerance there is that floor plus 1e-6; for the couplings the quotient with
    step 1e-4 (truncation ~1e-8) is held to 1e-6 as well."""
    print("case: trajectory 64^3 x 50 steps", flush=True)
    J, gth, gdir, fds = _grad_and_fd(64, 0.25, 50, 10, 8.0, 10.0, (1e-6, 1e-4))
    assert J > 0
    fd6, fdu6 = fds[1e-6]
    floor = np.spacing(J) / (2 * 1e-6 * np.abs(gth))
    assert np.all(np.abs(gth - fd6) / np.abs(gth) <= 1e-6 + floor), (gth, fd6, floor)
    assert gdir == pytest.approx(fdu6, rel=1e-6)
    fd4, _ = fds[1e-4]
    np.testing.assert_allclose(gth, fd4, rtol=1e-6)


def test_trajectory_gradient_vs_central_fd_256():
    """The large single-box workload: 256^3 two punctures, dx = M/16,
    lambda_gb = 0.2, g2 = 0.02, 20 RK4 steps with checkpoints every 2 steps
    (the checkpoint and stage buffers of a 3.9 GB state fit in HBM), J = sum
    over 8 < r < 10 of phi^2.  The adjoint's d J / d phi_0 . v (v smooth and
    random, on every stored cell) and d J / d lambda_gb are held against central
    differences with steps 1e-6 and 1e-4 respectively (relative 1e-6 plus the
    rounding floor ulp(J) / (2 h |J'|) of the difference quotient)."""
    print("case: trajectory 256^3 x 20 steps vs central differences", flush=True)
    p = I.default_params(lambda_gb=0.2, g2=0.02)
    n, dx, nsteps = 256, 1.0 / 16.0, 20
    dt = 0.25 * dx
    u0 = I.two_punctures(n, dx)
    mask = torch.from_numpy(I.shell_mask((n, n, n), dx, 8.0, 10.0)).to(DEV)
    ut = torch.from_numpy(u0).to(DEV)
    del u0
    traj = A.Trajectory(p, G.box_of(ut, dx), dt, nsteps, every=2)
    theta = torch.tensor([p["lambda_gb"], p["g2"]], dtype=torch.float64, requires_grad=True)
    u0t = ut.clone().requires_grad_(True)
    J = A.shell_phi2(A.Evolve.apply(theta, u0t, traj), mask)
    J.backward()
    gth = theta.grad.numpy().copy()
    X, Y, Z = I.coords((n, n, n), dx)
    rng = np.random.default_rng(3)
    v = torch.from_numpy(np.exp(-(X * X + Y * Y + Z * Z) / 40.0)
                         * rng.standard_normal(X.shape)).to(DEV)
    del X, Y, Z
    gdir = float((u0t.grad[I.IDX["phi"]] * v).sum())
    u0t.grad = None

    def Jof(th, phi_shift):
        with torch.no_grad():
            uin = ut.clone()
            uin[I.IDX["phi"]] += phi_shift
            un, _ = traj.forward(th, uin)
            return float(A.shell_phi2(un, mask))

    th0 = [p["lambda_gb"], p["g2"]]
    Jv = float(J.detach())
    assert Jv > 0
    h = 1e-6
    fd_u = (Jof(th0, h * v) - Jof(th0, -h * v)) / (2 * h)
    floor = np.spacing(Jv) / (2 * h * abs(gdir))
    assert abs(gdir - fd_u) <= (1e-6 + floor) * abs(gdir), (gdir, fd_u, floor)
    h = 1e-4
    fd_l = (Jof([th0[0] + h, th0[1]], 0.0) - Jof([th0[0] - h, th0[1]], 0.0)) / (2 * h)
    floor = np.spacing(Jv) / (2 * h * abs(gth[0]))
    assert abs(gth[0] - fd_l) <= (1e-6 + floor) * abs(gth[0]), (gth[0], fd_l, floor)


def test_trajectory_gradient_vs_oracle_tangent_cfg3_box():
    """64^3 box, dx = M/4, 10 RK4 steps: d J / d lambda_gb from the adjoint
    against the oracle's complex-step tangent through the same steps."""
    print("case: trajectory 64^3 x 10 steps vs oracle tangent", flush=True)
    n, dx, nsteps = 64, 0.25, 10
    p = I.default_params()
    dt = 0.25 * dx
    u0 = _cfg3(n, dx)
    maskn = I.shell_mask((n, n, n), dx, 5.0, 7.0)
    mask = torch.from_numpy(maskn).to(DEV)
    ut = torch.from_numpy(u0).to(DEV)
    traj = A.Trajectory(p, G.box_of(ut, dx), dt, nsteps, every=5)
    theta = torch.tensor([p["lambda_gb"], p["g2"]], dtype=torch.float64, requires_grad=True)
    J = A.shell_phi2(A.Evolve.apply(theta, ut.clone(), traj), mask)
    J.backward()
    ure, uim = O.rk4_cs(I.params_vector(p), np.array([H_CS, 0.0]), u0, np.zeros_like(u0), dx, dt, nsteps,
                        periodic=False)
    phi_re = I.interior(ure[I.IDX["phi"]][None])[0]
    phi_im = I.interior(uim[I.IDX["phi"]][None])[0] / H_CS
    tangent = float(np.sum((2 * phi_re * phi_im)[maskn]))
    assert float(theta.grad[0]) == pytest.approx(tangent, rel=1e-8)


@pytest.mark.parametrize("fd_order", [4.0, 6.0])
def test_trajectory_gradient_vs_oracle_tangent(fd_order):
    """Small box: the adjoint's dJ/dtheta and dJ/dphi0 . v against the oracle's
    complex-step tangent through the same RK4 steps (fourth- and sixth-order
    stencils)."""
    print("case: trajectory 16^3 x 6 steps vs oracle tangent, fd_order", fd_order, flush=True)
    p = I.default_params(lambda_gb=0.5, g2=0.05, fd_order=fd_order)
    n, dx, nsteps = 16, 0.5, 6
    dt = 0.25 * dx
    u0 = I.puncture((n, n, n), dx, phi_fn=I.shell_pulse(0.3, 2.0))
    maskn = I.shell_mask((n, n, n), dx, 2.0, 3.5)
    mask = torch.from_numpy(maskn).to(DEV)
    ut = torch.from_numpy(u0).to(DEV)
    traj = A.Trajectory(p, G.box_of(ut, dx), dt, nsteps, every=4)
    theta = torch.tensor([p["lambda_gb"], p["g2"]], dtype=torch.float64, requires_grad=True)
    u0t = ut.clone().requires_grad_(True)
    J = A.shell_phi2(A.Evolve.apply(theta, u0t, traj), mask)
    J.backward()
    rng = np.random.default_rng(1)
    v = np.zeros_like(u0)
    v[I.IDX["phi"]] = rng.standard_normal(u0.shape[1:])
    dth = np.array([0.6, -1.1])
    ure, uim = O.rk4_cs(I.params_vector(p), H_CS * dth, u0, H_CS * v, dx, dt, nsteps, periodic=False)
    phi_re = I.interior(ure[I.IDX["phi"]][None])[0]
    phi_im = I.interior(uim[I.IDX["phi"]][None])[0] / H_CS
    tangent = float(np.sum((2 * phi_re * phi_im)[maskn]))
    adj = float(theta.grad.numpy() @ dth + np.sum(u0t.grad.cpu().numpy() * v))
    assert adj == pytest.approx(tangent, rel=1e-9)
    # the forward J matches the oracle's too
    assert float(J.detach()) == pytest.approx(float(np.sum((phi_re ** 2)[maskn])), rel=1e-10)


@pytest.mark.parametrize("shift_advec", [0.0, 1.0])
def test_decoupled_vjp_dot_products_vs_oracle_tangent(shift_advec):
    """The decoupling limit (the scalar does not source the metric) has its
    own generated reverse: the right-hand side's and the RK4 step's VJPs
    against the oracle's complex-step tangent."""
    print("case: decoupled VJPs, shift_advec", shift_advec, flush=True)
    p = I.default_params(shift_advec=shift_advec, lambda_gb=0.3, g2=0.05, decoupled=1.0)
    dims, dx, dt = (11, 9, 7), 0.4, 0.1
    u = _state(dims, dx, 7)
    rng = np.random.default_rng(8)
    v = rng.standard_normal(u.shape)
    dth = np.array([0.5, -0.8])
    w = rng.standard_normal(u.shape) * _interior_mask(u.shape)
    _, jim = O.rhs_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx)
    lhs = np.sum(w * jim / H_CS * _interior_mask(u.shape))
    ut = torch.from_numpy(u).to(DEV)
    ubar = torch.zeros_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    box = G.box_of(ut, dx)
    G.rhs_vjp(G.make_params(p), box, ut, torch.from_numpy(w).to(DEV), ubar, tbar,
              G.alloc_workspace(G.vjp_workspace_bytes(box)))
    rhs = float(np.sum(ubar.cpu().numpy() * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)
    # and it is not the full theory's reverse
    ub_full = torch.zeros_like(ut)
    G.rhs_vjp(G.make_params(dict(p, decoupled=0.0)), box, ut, torch.from_numpy(w).to(DEV), ub_full,
              torch.zeros(2, dtype=torch.float64, device=DEV), G.alloc_workspace(G.vjp_workspace_bytes(box)))
    assert not torch.equal(ub_full, ubar)
    # one RK4 step
    w2 = rng.standard_normal(u.shape)
    _, uim = O.rk4_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx, dt, 1, periodic=False)
    lhs2 = np.sum(w2 * uim / H_CS)
    traj = A.Trajectory(p, box, dt, 1)
    P = traj._params([p["lambda_gb"], p["g2"]])
    bufs = [ut.clone() for _ in range(4)]
    traj.step(P, ut, traj._accbuf(ut.device), bufs)
    u2, u3, u4 = bufs[:3]
    ub2 = torch.empty_like(ut)
    tb2 = torch.zeros(2, dtype=torch.float64, device=DEV)
    G.rk4_step_vjp(P, box, dt, ut, u2, u3, u4, torch.from_numpy(w2).to(DEV), ub2, tb2,
                   G.alloc_workspace(G.step_vjp_workspace_bytes(box)))
    rhs2 = float(np.sum(ub2.cpu().numpy() * v) + tb2.cpu().numpy() @ dth)
    assert abs(lhs2 - rhs2) <= 1e-11 * max(abs(lhs2), 1.0), (lhs2, rhs2)
