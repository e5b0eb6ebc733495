"""The sixth-order scheme on boxes with four ghost layers on the GPU against
the oracle: there the advection stencil is of order 6 (offsets -2..4 and
mirror) and the Kreiss-Oliger term is the eighth difference, so the scheme
keeps order 6 with dissipation on.  One right-hand side on both split paths,
sampled cells of the 128^3 box, RK4 steps with periodic and frozen ghosts,
constraints, enforcement, the per-face boundary rules, the measured order,
and the refused paths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I
from parity_util import rel_err_per_field
from test_oracle_pins import _smooth_periodic_2d
from test_gpu_bc import FILL_CASES, FLAT, STEP_CASES

DEV = "cuda"
NG4 = 4


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    G.lib()


def _p6(**over):
    return I.default_params(fd_order=6.0, **over)


def gpu_rhs(params, u, dx, bc=G.BC_FROZEN, path=None):
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, bc, ng=NG4)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    out = torch.zeros_like(ut)
    p0 = G.get_stage_path()
    if path is not None:
        G.set_stage_path(path)
    try:
        G.rhs_eval(G.make_params(params), box, ut, out, ws)
        code, bits = G.status_fetch(ws)
    finally:
        G.set_stage_path(p0)
    return out.cpu().numpy(), code, bits


def _err(g, o):
    return rel_err_per_field(g, o, ng=NG4)


@pytest.mark.parametrize("shift_advec", [0.0, 1.0])
def test_rhs_parity_periodic_noise(shift_advec):
    print("case: sixth order, four ghosts, rhs noise 32^3, shift_advec", shift_advec, flush=True)
    p = _p6(shift_advec=shift_advec, lambda_gb=0.3, g2=0.05)
    u = I.flat_noise_pulse(32, 0.25, seed=0, ng=NG4)
    u[I.IDX["shift1"]] += 1e-3 * np.sin(np.arange(u.shape[-1]))[None, None, :]
    u[I.IDX["shift2"]] -= 1e-3 * np.cos(np.arange(u.shape[-2]))[None, :, None]
    u = I.wrap_ghosts(u, NG4)
    o, fo = O.rhs(I.params_vector(p), u, 0.25, ng=NG4)
    assert fo == 0
    for path in (0, 2):
        g, code, bits = gpu_rhs(p, u, 0.25, G.BC_PERIODIC, path)
        assert code == 0 and bits == 0
        e = _err(g, o)
        assert e.max() <= 1e-12, (path, dict(zip(I.FIELDS, e)))
        # the ghosts of the result are not written
        assert np.all(g[:, :NG4] == 0.0) and np.all(g[..., -NG4:] == 0.0)


def test_rhs_parity_puncture_ragged():
    print("case: sixth order, four ghosts, rhs puncture 21x17x13", flush=True)
    p = _p6(lambda_gb=0.3, g2=0.05)
    dims, dx = (21, 17, 13), 0.3
    u = I.puncture(dims, dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0), ng=NG4)
    rng = np.random.default_rng(4)
    u[I.IDX["shift1"]:I.IDX["shift3"] + 1] += 0.01 * rng.standard_normal(u[19:22].shape)
    u[I.IDX["K"]] += 0.01 * rng.standard_normal(u[7].shape)
    o, _ = O.rhs(I.params_vector(p), u, dx, ng=NG4)
    g, code, _ = gpu_rhs(p, u, dx)
    assert code == 0
    e = _err(g, o)
    assert e.max() <= 1e-12, dict(zip(I.FIELDS, e))
    # the same interior on three ghost layers gives another result (advection
    # and dissipation differ)
    u3 = u[:, 1:-1, 1:-1, 1:-1].copy()
    ut3 = torch.from_numpy(u3).to(DEV)
    box3 = G.box_of(ut3, dx)
    ws3 = G.alloc_workspace(G.workspace_bytes(box3))
    out3 = torch.zeros_like(ut3)
    G.rhs_eval(G.make_params(p), box3, ut3, out3, ws3)
    g3 = out3.cpu().numpy()
    assert np.abs(I.interior(g3) - I.interior(g, NG4)).max() > 1e-8


def test_rhs_parity_full_size_sampled():
    print("case: sixth order, four ghosts, rhs single puncture 128^3 sampled", flush=True)
    p = _p6(shift_advec=1.0)
    u = I.single_puncture(128, 1.0 / 8.0, ng=NG4)
    rng = np.random.default_rng(31)
    u[I.IDX["shift1"]:I.IDX["shift3"] + 1] += 0.01 * rng.standard_normal(u[19:22].shape)
    g, code, _ = gpu_rhs(p, u, 1.0 / 8.0)
    assert code == 0
    cells = rng.integers(0, 128, size=(2000, 3))
    cells = np.concatenate([cells, np.array([[63, 63, 63], [64, 64, 64], [0, 0, 0], [127, 127, 127]])])
    o, _ = O.rhs_cells(I.params_vector(p), u, 1.0 / 8.0, cells, ng=NG4)
    gs = g[:, cells[:, 2] + NG4, cells[:, 1] + NG4, cells[:, 0] + NG4].T
    num = np.abs(gs - o).max(axis=0)
    den = np.abs(o).max(axis=0)
    den = np.where(den > 0, den, den.max())
    assert (num / den).max() <= 1e-12, dict(zip(I.FIELDS, num / den))


@pytest.mark.parametrize("periodic", [True, False])
def test_rk4_ten_steps(periodic):
    print("case: sixth order, four ghosts, 10 RK4 steps 24^3, periodic", periodic, flush=True)
    p = _p6(lambda_gb=0.2, g2=0.02, shift_advec=1.0)
    if periodic:
        u = I.flat_noise_pulse(24, 0.25, seed=2, noise=1e-4, ng=NG4)
        bc = G.BC_PERIODIC
    else:
        u = I.single_puncture(24, 0.25, ng=NG4)
        bc = G.BC_FROZEN
    o, flags = O.rk4(I.params_vector(p), u, 0.25, 0.0625, 10, periodic=periodic, ng=NG4)
    assert flags == 0
    ut = torch.from_numpy(u).to(DEV)
    st = G.Stepper(G.make_params(p), G.box_of(ut, 0.25, bc, ng=NG4), ut, 0.0625)
    for _ in range(10):
        st.step()
    assert st.status() == (0, 0)
    e = rel_err_per_field(st.u.cpu().numpy(), o, interior=False)
    assert e.max() <= 1e-10, dict(zip(I.FIELDS, e))


def test_fill_periodic_four_layers():
    u = I.flat_noise_pulse(9, 0.5, seed=3, noise=1e-3, ng=NG4)
    u[:, :NG4] = 0.0
    u[..., -NG4:] = 0.0
    ut = torch.from_numpy(u).to(DEV)
    G.fill_periodic(G.box_of(ut, 0.5, G.BC_PERIODIC, ng=NG4), ut)
    assert np.array_equal(ut.cpu().numpy(), I.wrap_ghosts(u, NG4))


def test_constraints_and_enforcement():
    print("case: sixth order, four ghosts, constraints and enforcement", flush=True)
    p = _p6(lambda_gb=0.3, g2=0.05)
    dx = 0.3
    u = I.puncture((21, 17, 13), dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0), ng=NG4)
    ho, mo = O.constraints(I.params_vector(p), u, dx, ng=NG4)
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, ng=NG4)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    hg, mg = G.constraints(G.make_params(p), box, ut, ws)
    hg, mg = hg.cpu().numpy(), mg.cpu().numpy()
    assert np.abs(hg - ho).max() <= 1e-12 * np.abs(ho).max()
    for d in range(3):
        assert np.abs(mg[d] - mo[d]).max() <= 1e-12 * np.abs(mo[d]).max()
    rng = np.random.default_rng(8)
    v = u.copy()
    v[1:14] += 0.05 * rng.standard_normal(v[1:14].shape)
    v[0] -= 0.5
    q = dict(p, enforce=1, chi_min=1e-4, lapse_min=1e-3)
    oe = O.enforce(v, 1e-4, 1e-3, ng=NG4)
    vt = torch.from_numpy(v).to(DEV)
    G.enforce(G.make_params(q), G.box_of(vt, dx, ng=NG4), vt)
    e = rel_err_per_field(vt.cpu().numpy(), oe, interior=False)
    assert e.max() <= 1e-14, dict(zip(I.FIELDS, e))
    # ghosts untouched
    assert np.array_equal(vt.cpu().numpy()[:, :NG4], v[:, :NG4])


@pytest.mark.parametrize("variant", ["decoupled", "general_coupling"])
def test_rhs_parity_other_theories(variant):
    """The decoupling limit and the general coupling run their own pointwise
    code; on four ghost layers they take the same moved state."""
    print("case: sixth order, four ghosts, rhs", variant, flush=True)
    over = dict(decoupled=1.0) if variant == "decoupled" else dict(lambda_lin=0.15, beta=1.5)
    p = _p6(lambda_gb=0.3, g2=0.05, shift_advec=1.0, **over)
    dims, dx = (19, 13, 11), 0.3
    u = I.puncture(dims, dx, centre=(0.2, 0.1, -0.3), phi_fn=I.shell_pulse(0.1, 2.0), ng=NG4)
    rng = np.random.default_rng(12)
    u[I.IDX["shift1"]:I.IDX["shift3"] + 1] += 0.01 * rng.standard_normal(u[19:22].shape)
    o, _ = O.rhs(I.params_vector(p), u, dx, ng=NG4)
    g, code, _ = gpu_rhs(p, u, dx)
    assert code == 0
    e = _err(g, o)
    assert e.max() <= 1e-12, dict(zip(I.FIELDS, e))


def test_energy_and_coupling_diagnostics():
    print("case: sixth order, four ghosts, energy and coupling diagnostics", flush=True)
    p = _p6(lambda_gb=0.3, g2=0.05)
    dx = 0.3
    u = I.puncture((17, 15, 13), dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0), ng=NG4)
    u[I.IDX["Pi"]] += 0.02
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, ng=NG4)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    for got, want in ((G.energy_densities(G.make_params(p), box, ut, ws), O.energy_densities(I.params_vector(p), u, dx, ng=NG4)),
                      (G.coupling_diagnostics(G.make_params(p), box, ut, ws), O.coupling(I.params_vector(p), u, dx, ng=NG4))):
        got = got.cpu().numpy()
        for q in range(want.shape[0]):
            assert np.abs(got[q] - want[q]).max() <= 1e-12 * max(np.abs(want[q]).max(), 1e-300), q


def test_gpu_rhs_converges_at_sixth_order_with_dissipation():
    """With four ghost layers the GPU right-hand side of smooth periodic data
    converges at sixth order with the shift and the dissipation on."""
    print("case: sixth order, four ghosts, spatial convergence on the GPU", flush=True)
    L = 8.0
    p = _p6(ko_sigma=0.3, lambda_gb=0.2, g2=0.05)
    modes = [(0, 0), (1, 0), (1, 2), (2, -1)]
    coefs = []
    for n in (16, 32, 64):
        u, dx = _smooth_periodic_2d(n, L, True, NG4)
        r, code, _ = gpu_rhs(p, u, dx, G.BC_PERIODIC)
        assert code == 0
        X, Y, _ = I.coords((n, n, 4), dx, ng=NG4)
        x, y = I.interior(X[None], NG4)[0], I.interior(Y[None], NG4)[0]
        ri = I.interior(r, NG4)
        kk = 2 * np.pi / L
        coefs.append(np.array([[np.mean(ri[f] * np.exp(-1j * kk * (m * x + l * y))) for (m, l) in modes]
                               for f in range(27)]))
    c = np.array(coefs)
    d1 = np.abs(c[0] - c[1]).max(axis=1)
    d2 = np.abs(c[1] - c[2]).max(axis=1)
    live = d2 > 1e-12 * np.abs(c[2]).max()
    order_f = np.log2(d1[live] / d2[live])
    assert 5.6 < np.median(order_f) < 6.4, order_f


@pytest.mark.parametrize("dims", [(5, 7, 4), (16, 9, 11)])
@pytest.mark.parametrize("case", sorted(FILL_CASES))
def test_bc_fill_bitwise_against_oracle(case, dims):
    print("case: four ghosts, fill", case, dims, flush=True)
    bc = FILL_CASES[case]
    rng = np.random.default_rng(5)
    u = rng.standard_normal((I.NF, dims[2] + 2 * NG4, dims[1] + 2 * NG4, dims[0] + 2 * NG4))
    want = O.fill_bc(u, 0.25, bc, ng=NG4)
    ut = torch.from_numpy(u).to(DEV)
    G.bc_fill(G.make_bc(**bc), G.box_of(ut, 0.25, ng=NG4), ut)
    assert np.array_equal(ut.cpu().numpy(), want)


def test_bc_ghost_rhs_against_oracle():
    print("case: four ghosts, radiative ghost rhs", flush=True)
    dims, h = (12, 9, 7), 0.25
    origin = (-0.5 * dims[0] * h + 0.5 * h, -0.5 * dims[1] * h + 0.5 * h + 0.1, -0.5 * dims[2] * h + 0.5 * h)
    X, Y, Z = I.coords(dims, h, ng=NG4)
    rng = np.random.default_rng(2)
    u = I.set_flat(I.empty_state(dims, NG4))
    for f in range(I.NF):
        a = 0.1 * rng.standard_normal(4)
        u[f] += a[0] * np.sin(0.3 * X + a[1]) * np.cos(0.2 * Y - a[2]) + a[3] * np.exp(-0.01 * (X * X + Z * Z))
    bc = dict(rules=["sommerfeld", "sommerfeld", "reflective", "sommerfeld", "frozen", "sommerfeld"],
              centre=(0.05, -0.02, 0.01), speed=0.5 + rng.random(I.NF), asymptote=FLAT, origin=origin)
    want = O.ghost_rhs(u, h, bc, ng=NG4)
    ut = torch.from_numpy(u).to(DEV)
    got = G.bc_ghost_rhs(G.make_bc(**bc), G.box_of(ut, h, origin=origin, ng=NG4), ut).cpu().numpy()
    scale = np.abs(want).max(axis=(1, 2, 3))
    err = np.abs(got - want).max(axis=(1, 2, 3)) / scale
    assert err.max() <= 1e-13, err


@pytest.mark.parametrize("case", sorted(STEP_CASES))
def test_rk4_steps_with_faces_against_oracle(case):
    print("case: four ghosts, RK4 with faces", case, flush=True)
    dims, h, dt, nsteps = (14, 12, 10), 0.3, 0.075, 3
    origin = (-0.5 * dims[0] * h + 0.5 * h, -0.5 * dims[1] * h + 0.5 * h, -0.5 * dims[2] * h + 0.5 * h)
    u = I.puncture(dims, h, centre=(0.0, 0.0, 0.0), phi_fn=I.shell_pulse(0.1, 1.5), ng=NG4)
    bc = dict(STEP_CASES[case], centre=(0.01, 0.02, -0.03), speed=np.where(np.arange(I.NF) == 18, 2 ** 0.5, 1.0),
              asymptote=FLAT, origin=origin)
    p = _p6(lambda_gb=0.2, g2=0.05)
    u = O.fill_bc(u, h, bc, ng=NG4)
    want, flags = O.rk4_bc(I.params_vector(p), u, h, dt, nsteps, bc, ng=NG4)
    assert flags == 0
    ut = torch.from_numpy(u).to(DEV)
    st = G.StepperBC(G.make_params(p), G.box_of(ut, h, origin=origin, ng=NG4), ut, dt, G.make_bc(**bc))
    for _ in range(nsteps):
        st.step()
    assert st.status() == (0, 0)
    e = rel_err_per_field(st.u.cpu().numpy(), want, interior=False)
    assert e.max() <= 1e-10, dict(zip(I.FIELDS, e))


H_CS = 1e-30


def _vjp_state(dims, dx, seed, amp=0.02):
    u = I.puncture(dims, dx, centre=(0.7, -0.4, 0.3), phi_fn=I.shell_pulse(0.2, 1.5), ng=NG4)
    rng = np.random.default_rng(seed)
    u += amp * rng.standard_normal(u.shape) * (np.abs(u) + 0.1)
    u[I.IDX["lapse"]] = np.abs(u[I.IDX["lapse"]]) + 0.2
    u[I.IDX["chi"]] = np.abs(u[I.IDX["chi"]]) + 0.1
    return u


@pytest.mark.parametrize("shift_advec", [0.0, 1.0])
def test_rhs_vjp_dot_product_vs_oracle_tangent(shift_advec):
    """<w, J v + J_theta dth> from the oracle's complex step equals
    <J^T w, v> + <J_theta^T w, dth> from the GPU adjoint, on four ghost layers
    (the transposes of the seven-point biased stencils and the eighth
    difference)."""
    print("case: four ghosts, RHS VJP 11x9x7 shift_advec", shift_advec, flush=True)
    p = _p6(shift_advec=shift_advec, lambda_gb=0.3, g2=0.05)
    dims, dx = (11, 9, 7), 0.4
    u = _vjp_state(dims, dx, 1)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(u.shape)
    dth = np.array([0.7, -0.4])
    inner = np.zeros(u.shape, bool)
    inner[:, NG4:-NG4, NG4:-NG4, NG4:-NG4] = True
    w = rng.standard_normal(u.shape) * inner
    _, jim = O.rhs_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx, ng=NG4)
    lhs = np.sum(w * jim / H_CS * inner)
    ut = torch.from_numpy(u).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    ubar = torch.zeros_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    box = G.box_of(ut, dx, ng=NG4)
    G.rhs_vjp(G.make_params(p), box, ut, wt, ubar, tbar, G.alloc_workspace(G.vjp_workspace_bytes(box)))
    ub = ubar.cpu().numpy()
    rhs = float(np.sum(ub * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)
    # cotangents reach the fourth ghost layer (the eighth difference and the
    # biased stencils read it) and nothing beyond the stencils' reach
    assert np.abs(ub[:, 0, NG4:-NG4, NG4:-NG4]).max() > 0


def test_rk4_step_vjp_vs_oracle_tangent():
    print("case: four ghosts, RK4 step VJP 10x8x9", flush=True)
    p = _p6(lambda_gb=0.3, g2=0.05, shift_advec=1.0)
    dims, dx, dt = (10, 8, 9), 0.4, 0.1
    u = _vjp_state(dims, dx, 5, amp=0.01)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(u.shape)
    dth = np.array([-0.3, 0.9])
    w = rng.standard_normal(u.shape)
    _, uim = O.rk4_cs(I.params_vector(p), H_CS * dth, u, H_CS * v, dx, dt, 1, periodic=False, ng=NG4)
    lhs = np.sum(w * uim / H_CS)
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, ng=NG4)
    P = G.make_params(p)
    acc = torch.zeros((I.NF, box.nx * box.ny * box.nz), dtype=torch.float64, device=DEV)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    u2, u3, u4, un = (ut.clone() for _ in range(4))
    G.rk4_stage(P, box, 1, dt, ut, ut, u2, acc, ws)
    G.rk4_stage(P, box, 2, dt, ut, u2, u3, acc, ws)
    G.rk4_stage(P, box, 3, dt, ut, u3, u4, acc, ws)
    ubar = torch.empty_like(ut)
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    wsv = G.alloc_workspace(G.step_vjp_workspace_bytes(box))
    G.rk4_step_vjp(P, box, dt, ut, u2, u3, u4, torch.from_numpy(w).to(DEV), ubar, tbar, wsv)
    rhs = float(np.sum(ubar.cpu().numpy() * v) + tbar.cpu().numpy() @ dth)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0), (lhs, rhs)


def test_four_ghost_layers_refused_elsewhere():
    u = torch.from_numpy(I.single_puncture(12, 0.25, ng=NG4)).to(DEV)
    box = G.box_of(u, 0.25, ng=NG4)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    out = torch.zeros_like(u)
    # the fourth-order scheme
    with pytest.raises(G.GrfError) as e:
        G.rhs_eval(G.make_params(I.default_params()), box, u, out, ws)
    assert e.value.code == 7
    p = G.make_params(_p6())
    with pytest.raises((G.GrfError, ValueError)):
        G.Batch(p, [box], [u], [0.01])
    # the adjoint of the fourth-order scheme
    tbar = torch.zeros(2, dtype=torch.float64, device=DEV)
    with pytest.raises(G.GrfError) as e:
        G.rhs_vjp(G.make_params(I.default_params()), box, u, torch.zeros_like(u), torch.zeros_like(u), tbar,
                  G.alloc_workspace(G.vjp_workspace_bytes(box)))
    assert e.value.code == 7
    # a reflective face needs as many interior cells as there are ghost layers
    thin = torch.from_numpy(I.single_puncture(3, 0.25, ng=NG4)).to(DEV)
    with pytest.raises(G.GrfError) as e:
        G.bc_fill(G.make_bc(["reflective"] * 6), G.box_of(thin, 0.25, ng=NG4), thin)
    assert e.value.code == 1
