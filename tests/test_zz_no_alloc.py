"""grf_rk4_stage_static (no allocation, no workspace: the derivative records in
the library's own device array) against grf_rk4_stage (caller's workspace),
through the C-ABI: the same bits, on two boxes in a row, the second smaller
than the first, so that the second call runs over the first one's leftovers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    G.lib()


def _step_both(p, u, dx, dt, bc, ng=3):
    """One RK4 step (four stages) through each entry point from the same state."""
    P = G.make_params(p)
    ut = torch.from_numpy(u).to(DEV)
    box = G.box_of(ut, dx, bc, ng=ng)
    n = box.nx * box.ny * box.nz
    out = []
    for static in (False, True):
        ua, ub = ut.clone(), ut.clone()
        acc = torch.zeros((I.NF, n), dtype=torch.float64, device=DEV)
        if static:
            status = torch.zeros(1, dtype=torch.float64, device=DEV)
            G.status_clear(status)
            run = lambda s, us, un: G.rk4_stage_static(P, box, s, dt, ut, us, un, acc, status)
        else:
            status = G.alloc_workspace(G.workspace_bytes(box))
            run = lambda s, us, un: G.rk4_stage(P, box, s, dt, ut, us, un, acc, status)
        run(1, ut, ua)
        run(2, ua, ub)
        run(3, ub, ua)
        run(4, ua, ub)
        torch.cuda.synchronize()
        assert G.status_fetch(status) == (0, 0)
        out.append((ub.clone(), acc.clone()))
    return out


def test_static_stage_matches_workspace_stage_two_calls():
    # first call: 96 x 96 x 20 cells, several z-slabs of the 128 MiB array
    # (9 planes of 9,216 cells per slab)
    print("case: static-scratch stage, 96x96x20 puncture then 24x20x13 periodic noise", flush=True)
    p = I.default_params()
    u = I.puncture((96, 96, 20), 0.125, centre=(0.3, -0.2, 0.1), phi_fn=I.shell_pulse(0.1, 4.0))
    (a, acc_a), (b, acc_b) = _step_both(p, u, 0.125, 0.03125, G.BC_FROZEN)
    assert torch.equal(a, b) and torch.equal(acc_a, acc_b)
    # second call, smaller: one slab, periodic ghosts filled by the call
    print("case: static-scratch stage, second call 24x20x13", flush=True)
    u2 = I.set_flat(I.empty_state((24, 20, 13)))
    rng = np.random.default_rng(3)
    u2[:, 3:-3, 3:-3, 3:-3] += rng.uniform(-1e-6, 1e-6, (I.NF, 13, 20, 24))
    u2 = I.wrap_ghosts(u2)
    (c, acc_c), (d, acc_d) = _step_both(I.default_params(shift_advec=1.0), u2, 0.25, 0.0625, G.BC_PERIODIC)
    assert torch.equal(c, d) and torch.equal(acc_c, acc_d)


def test_static_stage_sixth_order_four_ghosts():
    print("case: static-scratch stage, sixth order on four ghost layers, 40x33x27", flush=True)
    p = I.default_params(fd_order=6)
    u = I.puncture((40, 33, 27), 0.25, centre=(0.1, 0.2, -0.1), phi_fn=I.shell_pulse(0.1, 2.0), ng=4)
    (a, acc_a), (b, acc_b) = _step_both(p, u, 0.25, 0.0625, G.BC_FROZEN, ng=4)
    assert torch.equal(a, b) and torch.equal(acc_a, acc_b)
