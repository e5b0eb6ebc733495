"""Sixth-order stencils on the GPU against the oracle: one right-hand side on
both split paths, sampled cells of the 128^3 box, RK4 steps, the constraint
diagnostics, the measured spatial order, and the refused paths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I
from parity_util import rel_err_per_field
from test_oracle_pins import _smooth_periodic_2d

DEV = "cuda"


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
    box = G.box_of(ut, dx, bc)
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


@pytest.mark.parametrize("ng", [3, 4])
@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 5, 1), (1, 3, 7), (70, 2, 3)])
def test_rhs_parity_degenerate_boxes(dims, ng):
    """Sixth-order stencils on boxes of a single cell, one or two cells
    thick, or with a row longer than a wave (frozen ghosts, three or four
    layers): one right-hand side within 1e-12 of the oracle on both paths."""
    print("case: sixth order rhs, degenerate box", dims, "ng", ng, flush=True)
    p = _p6(shift_advec=1.0, lambda_gb=0.3, g2=0.05)
    dx = 0.3
    u = I.puncture(dims, dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0), ng=ng)
    rng = np.random.default_rng(8)
    u[I.IDX["shift1"]:I.IDX["shift3"] + 1] += 0.05 * rng.standard_normal(u[19:22].shape)
    o, fo = O.rhs(I.params_vector(p), u, dx, ng=ng)
    assert fo == 0
    for path in (0, 2):
        ut = torch.from_numpy(u).to(DEV)
        box = G.box_of(ut, dx, G.BC_FROZEN, ng=ng)
        ws = G.alloc_workspace(G.workspace_bytes(box))
        out = torch.zeros_like(ut)
        p0 = G.get_stage_path()
        G.set_stage_path(path)
        try:
            G.rhs_eval(G.make_params(p), box, ut, out, ws)
            code, bits = G.status_fetch(ws)
        finally:
            G.set_stage_path(p0)
        assert code == 0 and bits == 0
        e = rel_err_per_field(out.cpu().numpy(), o, ng=ng)
        assert e.max() <= 1e-12, (path, dict(zip(I.FIELDS, e)))


@pytest.mark.parametrize("shift_advec", [0.0, 1.0])
def test_rhs_parity_periodic_noise(shift_advec):
    print("case: sixth order rhs, noise 32^3, shift_advec", shift_advec, flush=True)
    p = _p6(shift_advec=shift_advec, lambda_gb=0.3, g2=0.05)
    u = I.flat_noise_pulse(32, 0.25, seed=0)
    u[I.IDX["shift1"]] += 1e-3 * np.sin(np.arange(u.shape[-1]))[None, None, :]
    u = I.wrap_ghosts(u)
    o, fo = O.rhs(I.params_vector(p), u, 0.25)
    assert fo == 0
    for path in (0, 2):
        g, code, bits = gpu_rhs(p, u, 0.25, G.BC_PERIODIC, path)
        assert code == 0 and bits == 0
        e = rel_err_per_field(g, o)
        assert e.max() <= 1e-12, (path, dict(zip(I.FIELDS, e)))


def test_rhs_parity_puncture_ragged():
    print("case: sixth order rhs, puncture 21x17x13 (ragged tiles)", flush=True)
    p = _p6(lambda_gb=0.3, g2=0.05)
    dims, dx = (21, 17, 13), 0.3
    u = I.puncture(dims, dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0))
    rng = np.random.default_rng(4)
    u[I.IDX["shift1"]:I.IDX["shift3"] + 1] += 0.01 * rng.standard_normal(u[19:22].shape)
    u[I.IDX["K"]] += 0.01 * rng.standard_normal(u[7].shape)
    o, _ = O.rhs(I.params_vector(p), u, dx)
    g, code, _ = gpu_rhs(p, u, dx)
    assert code == 0
    e = rel_err_per_field(g, o)
    assert e.max() <= 1e-12, dict(zip(I.FIELDS, e))
    # and it is not the fourth-order result
    g4, _, _ = gpu_rhs(I.default_params(lambda_gb=0.3, g2=0.05), u, dx)
    assert np.abs(g4 - g).max() > 1e-8


def test_rhs_parity_full_size_sampled():
    print("case: sixth order rhs, single puncture 128^3 sampled", flush=True)
    p = _p6()
    u = I.single_puncture(128, 1.0 / 8.0)
    g, code, _ = gpu_rhs(p, u, 1.0 / 8.0)
    assert code == 0
    rng = np.random.default_rng(29)
    cells = rng.integers(0, 128, size=(2000, 3))
    cells = np.concatenate([cells, np.array([[63, 63, 63], [64, 64, 64], [0, 0, 0], [127, 127, 127]])])
    o, _ = O.rhs_cells(I.params_vector(p), u, 1.0 / 8.0, cells)
    gs = g[:, cells[:, 2] + 3, cells[:, 1] + 3, cells[:, 0] + 3].T
    num = np.abs(gs - o).max(axis=0)
    den = np.abs(o).max(axis=0)
    den = np.where(den > 0, den, den.max())
    assert (num / den).max() <= 1e-12, dict(zip(I.FIELDS, num / den))


def test_rk4_ten_steps_puncture():
    print("case: sixth order, 10 RK4 steps 24^3 puncture", flush=True)
    p = _p6(lambda_gb=0.2, g2=0.02)
    u = I.single_puncture(24, 0.25)
    o, flags = O.rk4(I.params_vector(p), u, 0.25, 0.0625, 10, periodic=False)
    assert flags == 0
    ut = torch.from_numpy(u).to(DEV)
    st = G.Stepper(G.make_params(p), G.box_of(ut, 0.25), ut, 0.0625)
    for _ in range(10):
        st.step()
    assert st.status() == (0, 0)
    e = rel_err_per_field(st.u.cpu().numpy(), o, interior=False)
    assert e.max() <= 1e-10, dict(zip(I.FIELDS, e))


def test_constraints_parity():
    print("case: sixth order constraints", flush=True)
    p = _p6(lambda_gb=0.3, g2=0.05)
    dx = 0.3
    u = I.puncture((21, 17, 13), dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0))
    ho, mo = O.constraints(I.params_vector(p), u, dx)
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    hg, mg = G.constraints(G.make_params(p), box, ut, ws)
    hg, mg = hg.cpu().numpy(), mg.cpu().numpy()
    assert np.abs(hg - ho).max() <= 1e-12 * np.abs(ho).max()
    for d in range(3):
        assert np.abs(mg[d] - mo[d]).max() <= 1e-12 * np.abs(mo[d]).max()


def test_gpu_rhs_converges_at_sixth_order():
    """The GPU right-hand side of smooth periodic data (zero shift, no
    Kreiss-Oliger) converges at sixth order in its low Fourier modes."""
    print("case: sixth order spatial convergence on the GPU", flush=True)
    L = 8.0
    p = _p6(ko_sigma=0.0, lambda_gb=0.2, g2=0.05)
    modes = [(0, 0), (1, 0), (1, 2), (2, -1)]
    coefs = []
    for n in (16, 32, 64):
        u, dx = _smooth_periodic_2d(n, L, False)
        r, code, _ = gpu_rhs(p, u, dx, G.BC_PERIODIC)
        assert code == 0
        X, Y, _ = I.coords((n, n, 4), dx)
        x, y = I.interior(X[None])[0], I.interior(Y[None])[0]
        ri = I.interior(r)
        kk = 2 * np.pi / L
        coefs.append(np.array([[np.mean(ri[f] * np.exp(-1j * kk * (m * x + l * y))) for (m, l) in modes]
                               for f in range(27)]))
    c = np.array(coefs)
    d1 = np.abs(c[0] - c[1]).max(axis=1)
    d2 = np.abs(c[1] - c[2]).max(axis=1)
    live = d2 > 1e-12 * np.abs(c[2]).max()
    order_f = np.log2(d1[live] / d2[live])
    assert 5.6 < np.median(order_f) < 6.4, order_f


def test_unsupported_paths_are_refused():
    p = G.make_params(_p6())
    u = torch.from_numpy(I.single_puncture(16, 0.25)).to(DEV)
    box = G.box_of(u, 0.25)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    out = torch.zeros_like(u)
    with pytest.raises(G.GrfError):
        G.Batch(p, [box], [u], [0.01])
