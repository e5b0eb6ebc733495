"""The sub-box method of the multi-step parity tests on large boxes (CPU).

The GPU steps a whole box; the oracle steps only sub-boxes cut from the same
initial state with their outer layers frozen (parity_util.oracle_region_rk4).
This checks on a box small enough for the oracle to step whole that the
sub-box result equals the whole-box result bit for bit on the region, and that
the margin 3 (4n - 1) it keeps is needed: one cell less and a single step
already differs."""
import numpy as np

from oracle import oracle as O
from paper_2309_06225_amd import inputs as I
from parity_util import oracle_region_rk4


def test_subbox_reproduces_whole_box():
    O.build(force=False)
    p = I.default_params(lambda_gb=0.2, g2=0.02)
    n, dx = 40, 0.25
    dt = 0.25 * dx
    u = I.two_punctures(n, dx)
    pv = I.params_vector(p)
    for nsteps in (1, 2):
        whole, flags = O.rk4(pv, u, dx, dt, nsteps, periodic=False)
        assert flags == 0
        # an interior region, one at the low corner and one at the high
        # corner (their sub-boxes end at the box's own frozen ghosts)
        for r0, w in (((15, 16, 17), 6), ((0, 0, 0), 5), ((n - 4, n - 4, n - 4), 4)):
            got = oracle_region_rk4(O, pv, u, dx, dt, nsteps, r0, w)
            ref = whole[:, r0[2] + 3:r0[2] + 3 + w, r0[1] + 3:r0[1] + 3 + w, r0[0] + 3:r0[0] + 3 + w]
            assert np.array_equal(got, ref), (nsteps, r0)
    # one step, a margin of 8 instead of 9: the frozen layer shows
    whole, _ = O.rk4(pv, u, dx, dt, 1, periodic=False)
    a, w, m = 10, 6, 8
    sub = np.ascontiguousarray(u[:, a - m:a + w + m + 6, a - m:a + w + m + 6, a - m:a + w + m + 6])
    o, _ = O.rk4(pv, sub, dx, dt, 1, periodic=False)
    got = o[:, m + 3:m + 3 + w, m + 3:m + 3 + w, m + 3:m + 3 + w]
    ref = whole[:, a + 3:a + 3 + w, a + 3:a + 3 + w, a + 3:a + 3 + w]
    assert not np.array_equal(got, ref)
