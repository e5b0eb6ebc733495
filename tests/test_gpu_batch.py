"""Batched persistent launches against per-box launches and the oracle; graph
replays against eager steps; the tile autotuner."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2309_06225_amd import grf as G
from paper_2309_06225_amd import inputs as I
from parity_util import rel_err_per_field

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    G.lib()


def _make(boxes_spec, shift_advec=0.0):
    states, dts = I.amr_states(boxes_spec)
    p = I.default_params(shift_advec=shift_advec)
    boxes = [G.make_box(b["dims"], b["dx"]) for b in boxes_spec]
    return p, boxes, states, dts


SMALL = [dict(dims=(16, 24, 16), dx=0.5, centre=(3.0, 1.0, -2.0), level=1),
         dict(dims=(24, 16, 32), dx=0.25, centre=(-1.0, 0.5, 0.7), level=2),
         dict(dims=(16, 16, 16), dx=1.0, centre=(10.0, -6.0, 4.0), level=0),
         dict(dims=(19, 13, 11), dx=0.125, centre=(0.9, 0.4, -0.3), level=3)]


@pytest.mark.parametrize("shift_advec", [0.0, 1.0])
def test_batched_equals_per_box_bitwise(shift_advec):
    print("case: batch of 4 uneven boxes, shift_advec", shift_advec, flush=True)
    p, boxes, states, dts = _make(SMALL, shift_advec)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    for _ in range(2):
        A.step()
        B.step_perbox()
    torch.cuda.synchronize()
    for b in range(len(boxes)):
        assert torch.equal(A.state(b), B.state(b)), b
    assert A.status() == (0, 0)
    # one step each more, the batched one as four per-stage calls
    for stage in (1, 2, 3, 4):
        A.rk4_stage(stage)
    B.step_perbox()
    for b in range(len(boxes)):
        assert torch.equal(A.state(b), B.state(b)), b
    A.close()
    B.close()


TINY = [dict(dims=(1, 1, 1), dx=0.5, centre=(3.0, 1.0, -2.0), level=1),
        dict(dims=(1, 4, 2), dx=0.25, centre=(-1.0, 0.5, 0.7), level=2),
        dict(dims=(5, 3, 1), dx=1.0, centre=(10.0, -6.0, 4.0), level=0),
        dict(dims=(70, 2, 3), dx=0.125, centre=(0.9, 0.4, -0.3), level=3),
        dict(dims=(16, 24, 16), dx=0.5, centre=(2.0, -1.0, 1.0), level=1)]


def test_batched_degenerate_boxes():
    """Boxes of a single cell, one or two cells thick, or with a row longer
    than a wave of cells, batched with an ordinary one: bitwise the per-box
    launches on every stencil variant the batched form runs, and two steps
    within 1e-10 of the oracle."""
    print("case: batch with degenerate boxes", flush=True)
    p, boxes, states, dts = _make(TINY, 1.0)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    for v in (0, 5, 8):
        for b in range(len(boxes)):
            A.set_tile_variant(b, v)
        A.step()
        B.step_perbox()
        for b in range(len(boxes)):
            assert torch.equal(A.state(b), B.state(b)), (v, b)
    assert A.status() == (0, 0)
    A.close()
    B.close()
    C = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    C.step()
    C.step()
    for b, s in enumerate(states):
        o, _ = O.rk4(I.params_vector(p), s, TINY[b]["dx"], dts[b], 2, periodic=False)
        e = rel_err_per_field(C.state(b).cpu().numpy(), o, interior=False)
        assert e.max() <= 1e-10, (b, dict(zip(I.FIELDS, e)))
    C.close()


def test_per_stage_calls_equal_step_bitwise():
    """grf_batch_step is four grf_batch_rk4_stage calls: the same bits, and
    every step's state is back in the caller's tensor; a stage outside 1..4
    is refused."""
    p, boxes, states, dts = _make(SMALL, 1.0)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    for _ in range(3):
        A.step()
        for stage in (1, 2, 3, 4):
            B.rk4_stage(stage)
    for b in range(len(boxes)):
        assert A.state(b) is A.states[b]
        assert torch.equal(A.state(b), B.state(b)), b
    with pytest.raises(G.GrfError):
        A.rk4_stage(5)
    A.close()
    B.close()


def test_mixed_stencil_variants_bitwise():
    """Boxes of one batch on different stencil variants (tiled and z-marching,
    one launch per variant per stage) against per-box launches on the default
    variants; a variant the batched form cannot run is rejected."""
    p, boxes, states, dts = _make(SMALL)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    for b, v in enumerate((5, 8, 6, 4)):
        A.set_tile_variant(b, v)
        assert A.tile_variant(b) == v
    with pytest.raises(G.GrfError):
        A.set_tile_variant(0, 7)
    for _ in range(2):
        A.step()
        B.step_perbox()
    for b in range(len(boxes)):
        assert torch.equal(A.state(b), B.state(b)), b
    A.close()
    B.close()


def test_batched_matches_oracle():
    print("case: batch vs oracle, 2 steps", flush=True)
    p, boxes, states, dts = _make(SMALL[:3])
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    A.step()
    A.step()
    for b, s in enumerate(states):
        o, _ = O.rk4(I.params_vector(p), s, SMALL[b]["dx"], dts[b], 2, periodic=False)
        e = rel_err_per_field(A.state(b).cpu().numpy(), o, interior=False)
        assert e.max() <= 1e-10, (b, dict(zip(I.FIELDS, e)))
    A.close()


def test_graph_replays_match_eager():
    """Each replay is one step (four stages); eager work and synchronisations
    in between; every replay is checked against an eager batch."""
    print("case: hipGraph replays", flush=True)
    p, boxes, states, dts = _make(SMALL)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
        E = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
        torch.cuda.synchronize()
        graph = A.capture(stream)
        for rep in range(4):
            A.replay(graph, stream)
            E.step(stream)
            stream.synchronize()
            junk = torch.randn(1000, device=DEV).sum()  # unrelated eager work
            torch.cuda.synchronize()
            for b in range(len(boxes)):
                assert torch.equal(A.state(b), E.state(b)), (rep, b)
            del junk
    A.close()
    E.close()


def test_autotune_is_cached_and_result_independent():
    p, boxes, states, dts = _make(SMALL)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    A.autotune()
    v1 = [A.tile_variant(b) for b in range(len(boxes))]
    assert all(v in (0, 1, 2, 3, 4, 5, 6, 8) for v in v1)
    B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    assert [B.tile_variant(b) for b in range(len(boxes))] == v1  # cached per shape class
    C = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    A.step()
    A.step()
    C.step_perbox()
    C.step_perbox()
    for b in range(len(boxes)):
        assert torch.equal(A.state(b), C.state(b))
    for x in (A, B, C):
        x.close()


def test_amr_workload_boxes_match_oracle():
    """The 96-box workload after one batched step (autotuned, graph-free):
    every box against the oracle's step of the same box (about 20 s of oracle
    time on the host), every cell of the box, frozen ghosts included, within
    1e-10 relative per field (R12).  Boxes far from the puncture are
    ill-conditioned as the noise box is (R20): there K, A_ij and Theta are
    about 1e-6 after one step, formed from cancelling O(1) terms, and the
    double-precision oracle itself is off by up to ~1e-9 relative.  A box that
    misses 1e-10 against the double oracle is therefore held, field by field,
    to max(1e-10, 1.5 x the double oracle's own error) against the oracle run
    in long double."""
    print("case: 96 AMR boxes, every box against the oracle", flush=True)
    spec = I.amr_boxes()
    p, boxes, states, dts = _make(spec)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    A.autotune()
    A.step()
    torch.cuda.synchronize()
    assert A.status()[0] == 0
    pv = I.params_vector(p)
    worst, ill = {}, []
    for b in range(len(spec)):
        o, fo = O.rk4(pv, states[b], spec[b]["dx"], dts[b], 1, periodic=False)
        assert fo == 0
        g = A.state(b).cpu().numpy()
        e = rel_err_per_field(g, o, interior=False)
        lev = spec[b]["level"]
        worst[lev] = max(worst.get(lev, 0.0), float(e.max()))
        if e.max() <= 1e-10:
            continue
        ref, fl = O.rk4_ld(pv, states[b], spec[b]["dx"], dts[b], 1, periodic=False)
        assert fl == 0
        e_gpu = rel_err_per_field(g, ref, interior=False)
        e_orc = rel_err_per_field(o, ref, interior=False)
        bound = np.maximum(1e-10, 1.5 * e_orc)
        ill.append((b, f"{e_gpu.max():.2e}", f"{e_orc.max():.2e}"))
        assert np.all(e_gpu <= bound), (b, spec[b]["dims"], lev, {f: (e_gpu[i], bound[i]) for i, f in
                                                                  enumerate(I.FIELDS) if e_gpu[i] > bound[i]})
    print("largest relative error against the double oracle, per level:",
          {k: f"{v:.2e}" for k, v in sorted(worst.items())}, flush=True)
    print("boxes held against the long-double oracle (box, GPU error, double oracle's error):", ill, flush=True)
    A.close()


def test_amr_workload_batched_equals_per_box():
    """The 96-box workload: one batched step against per-box launches."""
    print("case: 96 AMR boxes", flush=True)
    spec = I.amr_boxes()
    p, boxes, states, dts = _make(spec)
    A = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(s).to(DEV) for s in states], dts)
    A.autotune()
    A.step()
    B.step_perbox()
    torch.cuda.synchronize()
    for b in range(len(boxes)):
        assert torch.equal(A.state(b), B.state(b)), b
    assert A.status()[0] == 0
    A.close()
    B.close()
