"""Per-face boundary rules on the GPU against the oracle: ghost refills
(bitwise), the radiative ghost right-hand side, RK4 steps with mixed faces,
reductions to the plain frozen and periodic steps, and the absorbing property
of Sommerfeld faces on an outgoing scalar pulse."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I
from parity_util import rel_err_per_field

DEV = "cuda"
NF = I.NF
FLAT = I.set_flat(I.empty_state((1, 1, 1)))[:, 3, 3, 3]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    G.lib()


def _dev(u):
    return torch.from_numpy(np.ascontiguousarray(u)).to(DEV)


def _random_state(dims, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((NF, dims[2] + 6, dims[1] + 6, dims[0] + 6))


FILL_CASES = {
    "reflective_odd_phi": dict(rules=["reflective"] * 6, parity_phi=-1),
    "mixed": dict(rules=["periodic", "periodic", "reflective", "reflective", "extrapolating", "extrapolating"],
                  extrap_order=1),
    "extrap0": dict(rules=["extrapolating"] * 6, extrap_order=0),
    "extrap1_frozen": dict(rules=["extrapolating", "frozen", "frozen", "extrapolating", "extrapolating", "sommerfeld"],
                           extrap_order=1),
}


def test_thin_boxes_fill_and_radiative_rhs():
    """Boxes one or two cells thick along an axis: periodic and order-0
    extrapolating faces there (the rules such a box allows), Sommerfeld on the
    others; fills bitwise and the radiative right-hand side at 1e-13 against
    the oracle; a reflective face on a thin axis is refused."""
    print("case: thin boxes", flush=True)
    for dims in ((1, 6, 5), (7, 2, 4), (3, 4, 1)):
        u = _random_state(dims, 9)
        thin = [a for a in range(3) if dims[a] <= 2][0]
        rules = ["sommerfeld"] * 6
        rules[2 * thin] = rules[2 * thin + 1] = "periodic"
        h = 0.25
        origin = (1.0, 2.0, -3.0)
        bc = dict(rules=rules, centre=(0.1, 0.2, 0.3), origin=origin, asymptote=np.zeros(NF))
        ut = _dev(u)
        box = G.box_of(ut, h, origin=origin)
        G.bc_fill(G.make_bc(**bc), box, ut)
        assert np.array_equal(ut.cpu().numpy(), O.fill_bc(u, h, bc)), dims
        want = O.ghost_rhs(u, h, bc)
        got = G.bc_ghost_rhs(G.make_bc(**bc), box, _dev(u)).cpu().numpy()
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), dims
        ex = dict(rules=["extrapolating"] * 6, extrap_order=0)
        ut = _dev(u)
        G.bc_fill(G.make_bc(**ex), box, ut)
        assert np.array_equal(ut.cpu().numpy(), O.fill_bc(u, h, ex)), dims
        refl = ["frozen"] * 6
        refl[2 * thin] = "reflective"
        with pytest.raises(G.GrfError):
            G.bc_fill(G.make_bc(refl), box, ut)


@pytest.mark.parametrize("dims", [(5, 7, 3), (16, 9, 11)])
@pytest.mark.parametrize("case", sorted(FILL_CASES))
def test_fill_bitwise_against_oracle(case, dims):
    print("case: fill", case, dims, flush=True)
    bc = FILL_CASES[case]
    u = _random_state(dims, 1)
    want = O.fill_bc(u, 0.25, bc)
    ut = _dev(u)
    box = G.box_of(ut, 0.25)
    G.bc_fill(G.make_bc(**bc), box, ut)
    assert np.array_equal(ut.cpu().numpy(), want)


def _sommerfeld_state(dims, h, seed):
    """Flat values plus smooth perturbations (the radiative rule sees smooth data)."""
    X, Y, Z = I.coords(dims, h)
    rng = np.random.default_rng(seed)
    u = I.set_flat(I.empty_state(dims))
    for f in range(NF):
        a = 0.1 * rng.standard_normal(4)
        u[f] += a[0] * np.sin(0.3 * X + a[1]) * np.cos(0.2 * Y - a[2]) + a[3] * np.exp(-0.01 * (X * X + Z * Z))
    return u


@pytest.mark.parametrize("dims", [(12, 9, 7), (128, 128, 128)])
def test_ghost_rhs_against_oracle(dims):
    print("case: radiative ghost rhs", dims, flush=True)
    h = 0.25 if dims[0] < 100 else 1.0 / 8
    origin = (-0.5 * dims[0] * h + 0.5 * h, -0.5 * dims[1] * h + 0.5 * h + 0.1, -0.5 * dims[2] * h + 0.5 * h)
    u = _sommerfeld_state(dims, h, 2)
    rng = np.random.default_rng(3)
    bc = dict(rules=["sommerfeld", "sommerfeld", "reflective", "sommerfeld", "frozen", "sommerfeld"],
              centre=(0.05, -0.02, 0.01), speed=0.5 + rng.random(NF), asymptote=FLAT, origin=origin)
    want = O.ghost_rhs(u, h, bc)
    ut = _dev(u)
    box = G.box_of(ut, h, origin=origin)
    got = G.bc_ghost_rhs(G.make_bc(**bc), box, ut).cpu().numpy()
    scale = np.abs(want).max(axis=(1, 2, 3))
    err = np.abs(got - want).max(axis=(1, 2, 3)) / scale
    assert err.max() <= 1e-13, err


STEP_CASES = {
    "mixed": dict(rules=["sommerfeld", "sommerfeld", "reflective", "reflective", "extrapolating", "extrapolating"],
                  extrap_order=1),
    "sommerfeld": dict(rules=["sommerfeld"] * 6),
    "periodic_x_frozen": dict(rules=["periodic", "periodic", "frozen", "sommerfeld", "extrapolating", "frozen"],
                              extrap_order=0),
}


@pytest.mark.parametrize("case", sorted(STEP_CASES))
def test_rk4_steps_against_oracle(case):
    print("case: RK4 with faces", case, flush=True)
    dims, h, dt, nsteps = (14, 12, 10), 0.3, 0.075, 3
    origin = (-0.5 * dims[0] * h + 0.5 * h, -0.5 * dims[1] * h + 0.5 * h, -0.5 * dims[2] * h + 0.5 * h)
    u = I.puncture(dims, h, centre=(0.0, 0.0, 0.0), phi_fn=I.shell_pulse(0.1, 1.5))
    bc = dict(STEP_CASES[case], centre=(0.01, 0.02, -0.03), speed=np.where(np.arange(NF) == 18, 2 ** 0.5, 1.0),
              asymptote=FLAT, origin=origin)
    p = I.default_params(lambda_gb=0.2, g2=0.05)
    u = O.fill_bc(u, h, bc)
    want, flags = O.rk4_bc(I.params_vector(p), u, h, dt, nsteps, bc)
    assert flags == 0
    ut = _dev(u)
    box = G.box_of(ut, h, origin=origin)
    st = G.StepperBC(G.make_params(p), box, ut, dt, G.make_bc(**bc))
    for _ in range(nsteps):
        st.step()
    assert st.status() == (0, 0)
    got = st.u.cpu().numpy()
    e = rel_err_per_field(got, want, interior=False)
    assert e.max() <= 1e-10, dict(zip(I.FIELDS, e))


@pytest.mark.parametrize("n", [24, 128])
def test_rk4_bc_reduces_to_plain_steps_bitwise(n):
    """All faces frozen: the same states as the plain frozen step; all faces
    periodic: the same states as the plain periodic step."""
    print("case: reductions", n, flush=True)
    p = G.make_params(I.default_params(lambda_gb=0.3, g2=0.05))
    u = I.flat_noise_pulse(n, 0.25, seed=1) if n < 100 else I.single_puncture(n, 1.0 / 8)
    h = 0.25 if n < 100 else 1.0 / 8
    for rule, boxbc in (("frozen", G.BC_FROZEN), ("periodic", G.BC_PERIODIC)):
        ua = _dev(O.fill_periodic(u) if rule == "periodic" else u)
        ub = ua.clone()
        A = G.Stepper(p, G.box_of(ua, h, boxbc), ua, 0.25 * h)
        B = G.StepperBC(p, G.box_of(ub, h), ub, 0.25 * h, G.make_bc([rule] * 6))
        for _ in range(2):
            A.step()
            B.step()
        torch.cuda.synchronize()
        assert torch.equal(A.u, B.u), rule


def test_sommerfeld_faces_absorb_an_outgoing_pulse():
    """A small scalar pulse on flat space leaves the box through Sommerfeld
    faces; with frozen faces it stays trapped.  After it has crossed the box,
    the scalar left inside is much smaller with Sommerfeld faces (measured:
    about a quarter of the trapped amplitude at h = 1/4, the second-order
    one-sided differences of the radiative rule reflect a little)."""
    print("case: absorbing faces", flush=True)
    n, h = 48, 0.25
    dt = 0.25 * h
    origin = (-0.5 * n * h + 0.5 * h,) * 3
    X, Y, Z = I.coords((n, n, n), h)
    u = I.set_flat(I.empty_state((n, n, n)))
    u[I.IDX["phi"]] = 1e-3 * np.exp(-(X * X + Y * Y + Z * Z) / 0.8)
    p = G.make_params(I.default_params())
    left = {}
    for rule in ("sommerfeld", "frozen"):
        bc = G.make_bc([rule] * 6, asymptote=FLAT, speed=np.where(np.arange(NF) == 18, 2 ** 0.5, 1.0))
        ut = _dev(u)
        st = G.StepperBC(p, G.box_of(ut, h, origin=origin), ut, dt, bc)
        for _ in range(int(round(10.0 / dt))):
            st.step()
        assert st.status() == (0, 0)
        v = st.u.cpu().numpy()
        left[rule] = np.abs(v[I.IDX["Pi"], 3:-3, 3:-3, 3:-3]).max()
    print("residual |Pi|:", left, flush=True)
    assert left["sommerfeld"] < 0.4 * left["frozen"], left
