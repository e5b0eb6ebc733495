"""GPU diagnostics against the oracle: the constraints, the fourth-order
self-convergence of the Hamiltonian constraint measured with the GPU path, and
the energy densities of the three terms of the scalar action."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I
from test_oracle_pins import _smooth_periodic

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    G.lib()


def gpu_constraints(p, u, dx, bc=G.BC_FROZEN):
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, bc)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    ham, mom = G.constraints(G.make_params(p), box, ut, ws)
    return ham.cpu().numpy(), mom.cpu().numpy()


def gpu_energy(p, u, dx, bc=G.BC_FROZEN):
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, bc)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    return G.energy_densities(G.make_params(p), box, ut, ws).cpu().numpy()


def _case(case):
    """noise32: the plain small periodic workload; puncture_ragged: a frozen
    puncture box whose extents are not multiples of any tile; thin and row:
    degenerate frozen boxes (one or two cells thick; a row longer than a
    wave of cells), with the same perturbations."""
    if case == "noise32":
        return I.flat_noise_pulse(32, 0.25, seed=0), 0.25, G.BC_PERIODIC
    dx, bc = 0.3, G.BC_FROZEN
    dims = {"puncture_ragged": (21, 17, 13), "thin": (1, 4, 2), "row": (70, 2, 3)}[case]
    u = I.puncture(dims, dx, centre=(0.4, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 2.0))
    rng = np.random.default_rng(4)
    u[I.IDX["K"]] += 0.01 * rng.standard_normal(u[7].shape)
    u[I.IDX["A11"]:I.IDX["A33"] + 1] += 0.01 * rng.standard_normal(u[8:14].shape)
    u[I.IDX["Pi"]] += 0.01 * rng.standard_normal(u[26].shape)
    return u, dx, bc


def _rel(g, o):
    return np.abs(g - o).max() / max(np.abs(o).max(), 1e-300)


def test_flat_space_constraints_exactly_zero():
    u = I.set_flat(I.empty_state((19, 13, 11)))
    ham, mom = gpu_constraints(I.default_params(), u, 0.25)
    assert np.all(ham == 0.0) and np.all(mom == 0.0)


@pytest.mark.parametrize("case", ["noise32", "puncture_ragged", "thin", "row"])
def test_constraints_match_oracle(case):
    print("case: constraints", case, flush=True)
    p = I.default_params(lambda_gb=0.3, g2=0.05)
    u, dx, bc = _case(case)
    ho, mo = O.constraints(I.params_vector(p), u, dx)
    hg, mg = gpu_constraints(p, u, dx, bc)
    assert _rel(hg, ho) <= 1e-12, _rel(hg, ho)
    for d in range(3):
        assert _rel(mg[d], mo[d]) <= 1e-12, (d, _rel(mg[d], mo[d]))


def test_hamiltonian_self_convergence_fourth_order_gpu():
    """Smooth periodic data varying along x, evolved to t = 1 with the GPU RK4
    path on 32, 64 and 128 cells; the lowest Fourier modes of the GPU
    Hamiltonian constraint converge at fourth order."""
    print("case: Hamiltonian self-convergence on the GPU", flush=True)
    L, T = 8.0, 1.0
    p = I.default_params()
    P = G.make_params(p)
    coefs = []
    for n in (32, 64, 128):
        u, dx = _smooth_periodic(n, L)
        dt = 0.25 * dx
        steps = int(round(T / dt))
        ut = torch.from_numpy(u).to(DEV)
        box = G.box_of(ut, dx, G.BC_PERIODIC)
        st = G.Stepper(P, box, ut, dt)
        for _ in range(steps):
            st.step()
        assert st.status() == (0, 0)
        ham, _ = G.constraints(P, box, st.u, st.ws)
        ham = ham.cpu().numpy()
        X, _, _ = I.coords((n, 4, 4), dx)
        x = I.interior(X[None])[0]
        coefs.append(np.array([np.mean(ham * np.exp(-1j * m * 2 * np.pi * x / L)) for m in (0, 1, 2)]))
    coefs = np.array(coefs)
    order = np.log2(np.abs(coefs[0] - coefs[1]) / np.abs(coefs[1] - coefs[2]))
    assert np.all(np.abs(order - 4.0) < 0.3), order


def test_flat_space_energy_densities_exactly_zero():
    u = I.set_flat(I.empty_state((19, 13, 11)))
    rho = gpu_energy(I.default_params(lambda_gb=0.3, g2=0.05), u, 0.25)
    assert np.all(rho == 0.0)


@pytest.mark.parametrize("case", ["noise32", "puncture_ragged", "thin", "row"])
def test_energy_densities_match_oracle(case):
    print("case: energy densities", case, flush=True)
    p = I.default_params(lambda_gb=0.3, g2=0.05)
    u, dx, bc = _case(case)
    ro = O.energy_densities(I.params_vector(p), u, dx)
    rg = gpu_energy(p, u, dx, bc)
    for q in range(3):
        assert np.abs(ro[q]).max() > 0.0, q
        assert _rel(rg[q], ro[q]) <= 1e-12, (q, _rel(rg[q], ro[q]))


def gpu_coupling(p, u, dx, bc=G.BC_FROZEN):
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, bc)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    return G.coupling_diagnostics(G.make_params(p), box, ut, ws).cpu().numpy()


@pytest.mark.parametrize("case", ["noise32", "puncture_ragged", "thin", "row"])
def test_coupling_diagnostics_match_oracle(case):
    print("case: Gauss-Bonnet invariant and weak-coupling indicators", case, flush=True)
    p = I.default_params(lambda_gb=0.3, g2=0.05)
    u, dx, bc = _case(case)
    co = O.coupling(I.params_vector(p), u, dx)
    cg = gpu_coupling(p, u, dx, bc)
    for q in range(4):
        assert np.abs(co[q]).max() > 0.0, q
        assert _rel(cg[q], co[q]) <= 1e-12, (q, _rel(cg[q], co[q]))


def test_coupling_diagnostics_full_size_sampled():
    """128^3 single puncture: GPU values at every cell, the oracle's at sampled
    cells (its box routine on a 3-cell-thick slab around each sampled plane)."""
    print("case: coupling diagnostics 128^3 sampled planes", flush=True)
    p = I.default_params(lambda_gb=0.2, g2=0.02)
    u = I.single_puncture(128, 1.0 / 8.0)
    cg = gpu_coupling(p, u, 1.0 / 8.0)
    for k in (0, 40, 64, 127):
        slab = u[:, k:k + 7, :, :]   # interior plane k and its 3 ghost planes either side
        co = O.coupling(I.params_vector(p), slab, 1.0 / 8.0)[:, 0]
        for q in range(4):
            assert _rel(cg[q, k], co[q]) <= 1e-12, (k, q, _rel(cg[q, k], co[q]))


def test_constraints_and_energy_full_size_sampled():
    """128^3 single puncture: GPU constraints and energy densities at every
    cell against the oracle on four planes (each a 1-cell-thick box with its
    three neighbour planes either side as ghosts)."""
    print("case: constraints and energy densities 128^3 sampled planes", flush=True)
    p = I.default_params(lambda_gb=0.2, g2=0.02)
    dx = 1.0 / 8.0
    u = I.single_puncture(128, dx)
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx)
    ws = G.alloc_workspace(G.workspace_bytes(box))
    P = G.make_params(p)
    ham, mom = G.constraints(P, box, ut, ws)
    rho = G.energy_densities(P, box, ut, ws)
    ham, mom, rho = ham.cpu().numpy(), mom.cpu().numpy(), rho.cpu().numpy()
    # relative per field: the error over the field's largest value in the box
    # (far from the puncture the constraints are ~1e-11, the result of
    # cancellation among much larger terms, so a plane's own maximum is no scale)
    s_ham = np.abs(ham).max()
    s_mom = np.abs(mom).max(axis=(1, 2, 3))
    s_rho = np.abs(rho).max(axis=(1, 2, 3))
    for k in (0, 40, 64, 127):
        slab = u[:, k:k + 7, :, :]
        ho, mo = O.constraints(I.params_vector(p), slab, dx)
        ro = O.energy_densities(I.params_vector(p), slab, dx)
        assert np.abs(ham[k] - ho[0]).max() <= 1e-12 * s_ham, k
        for d in range(3):
            assert np.abs(mom[d, k] - mo[d, 0]).max() <= 1e-12 * s_mom[d], (k, d)
        for q in range(3):
            assert np.abs(rho[q, k] - ro[q, 0]).max() <= 1e-12 * max(s_rho[q], 1e-300), (k, q)
