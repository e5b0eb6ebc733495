"""Benchmark of the 4dST/CCZ4 RHS + RK4 hot path on one MI355X.

Workload: one 128^3 box (3 frozen ghosts), dx = M/8, single non-spinning
puncture (M = 1) with the scalar shell phi = 0.1 exp(-(r-4)^2), couplings
lambda(phi) = 0.1 phi^2/4, g2 = 0.01, a = 0.2, b = 0.4, kappa = (0.1, 0, 1),
eta = 1, KO sigma = 0.3, dt = dx/4.  A step is one full RK4 step (4 stencil
stages + 4 pointwise/RK4 stages).  Inputs are resident in HBM before the timed
region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 cell-updates/s (4∂ST RHS+RK4 stage) at 1 GPU; adjoint/forward time ratio"
PEAK_FP64 = 78.6  # TFLOP/s, MI355X FP64 vector
PEAK_HBM = 8000.0  # GB/s


def source_hash() -> str:
    """Hash of the sources the staged pointwise kernel is compiled from (its
    device code, the generated algebra, the layout and its launcher)."""
    h = hashlib.sha256()
    for rel in ("paper_2309_06225_amd/csrc/kernels_fwd.h", "paper_2309_06225_amd/csrc/kernels_staged.h",
                "paper_2309_06225_amd/csrc/gen/gen_rhs_staged.inc", "paper_2309_06225_amd/csrc/gen/gen_layout.h",
                "paper_2309_06225_amd/csrc/tu_staged.hip"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            data = fh.read()
        # the flop counts the layout header also carries do not reach the kernel
        h.update(b"".join(l for l in data.splitlines(True) if not l.startswith(b"#define GRF_FLOPS_")))
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    if absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


# Algorithmic bytes of one fused RK4 stage per interior cell: read u_s, u_0 and
# the accumulator, write u_{s+1} and the accumulator, 27 FP64 fields each (halo
# re-reads and the derivative record between the two kernels are not
# algorithmic).
BYTES_STAGE = 5 * 27 * 8


def load_flops(case: str = "full_theory") -> dict:
    """Algorithmic flops per interior cell counted by the oracle's op-counting
    scalar, as stored in profiles/flops_per_cell.json (a CPU test keeps the file
    equal to the oracle's count)."""
    with open(os.path.join(ROOT, "profiles", "flops_per_cell.json")) as fh:
        return json.load(fh)["per_cell"][case]


def roofline_point(flops_cell: float, bytes_cell: float, cells: int, ms: float) -> dict:
    """One launch (or stage) of `cells` cells in `ms` milliseconds against
    min(FP64 peak, AI x HBM peak), AI = flops_cell / bytes_cell."""
    ai = flops_cell / bytes_cell
    achieved = flops_cell * cells / (ms * 1e-3) / 1e12
    peak = min(PEAK_FP64, ai * PEAK_HBM / 1000.0)
    return {"bound": "alu" if ai * PEAK_HBM / 1000.0 >= PEAK_FP64 else "hbm", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "flops_per_cell": flops_cell, "bytes_per_cell": bytes_cell,
            "intensity": ai, "ms": ms}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(params, u, dx, dt):
    """The CPU oracle, untuned, on one full RK4 step of the same box."""
    from oracle import oracle as O
    from paper_2309_06225_amd import inputs as I
    O.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    O.rk4(I.params_vector(params), u, dx, dt, 1, periodic=False)
    t = time.perf_counter() - t0
    ncell = (u.shape[1] - 6) * (u.shape[2] - 6) * (u.shape[3] - 6)
    out = {"value": ncell / t, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"one full RK4 step of the same {u.shape[3] - 6}^3 box ({t:.1f} s wall)"}
    # one core: one RK4 step of a 4-plane slab of the same box (its neighbouring
    # planes as frozen ghosts)
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        mid = u.shape[1] // 2
        slab = np.ascontiguousarray(u[:, mid - 5:mid + 5])
        t0 = time.perf_counter()
        O.rk4(I.params_vector(params), slab, dx, dt, 1, periodic=False)
        t1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        nslab = (slab.shape[1] - 6) * (slab.shape[2] - 6) * (slab.shape[3] - 6)
        out["single_core"] = {"value": nslab / t1, "cores": 1,
                              "sample": f"one RK4 step of a {slab.shape[3] - 6}x{slab.shape[2] - 6}x4 slab "
                                        f"of the same box ({t1:.1f} s wall)"}
    except OSError:
        pass
    return out


def adjoint_ratio(torch, G, I):
    """64^3 puncture box, dx = M/4, 50 RK4 steps, checkpoints every 10:
    (backward incl. recomputation) / forward time, J = sum_{8<r<10} phi^2."""
    from paper_2309_06225_amd import adjoint as A
    n, dx, nsteps = 64, 0.25, 50
    p = I.default_params()
    u0 = torch.from_numpy(I.single_puncture(n, dx)).to("cuda")
    mask = torch.from_numpy(I.shell_mask((n, n, n), dx, 8.0, 10.0)).to("cuda")
    traj = A.Trajectory(p, G.box_of(u0, dx), 0.25 * dx, nsteps, every=10)
    theta = torch.tensor([p["lambda_gb"], p["g2"]], dtype=torch.float64, requires_grad=True)
    times = []
    for rep in range(2):  # the first repetition allocates the buffers
        theta.grad = None
        x = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = A.shell_phi2(A.Evolve.apply(theta, x, traj), mask)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    f, b = times[-1]
    # the same with every stencil stage on the 128-wide column (the single-box
    # default for this 64-wide box before narrow boxes got the 16x16 column):
    # a slower forward, so a lower ratio at a higher cost
    v0 = G.get_tile_variant()
    G.set_tile_variant(9)
    try:
        theta.grad = None
        x = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = A.shell_phi2(A.Evolve.apply(theta, x, traj), mask)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    finally:
        G.set_tile_variant(v0)
    wide = {"forward_s": t1 - t0, "backward_s": t2 - t1, "ratio": (t2 - t1) / (t1 - t0)}
    # one more backward, not timed, with the kernels of each right-hand-side
    # VJP timed by HIP events: the whole VJP and its reverse pointwise kernel
    theta.grad = None
    x = u0.clone().requires_grad_(True)
    J = A.shell_phi2(A.Evolve.apply(theta, x, traj), mask)
    G.prof_begin(4 * nsteps)
    J.backward()
    torch.cuda.synchronize()
    prof = G.prof_end()
    vjp_ms, vjp_n = prof["vjp"]
    pt_ms, pt_n = prof["vjp_point"]
    pt_avg = pt_ms / max(pt_n, 1)
    flops = G.flops_per_cell(2)
    tflops = flops * n ** 3 / (pt_avg * 1e-3) / 1e12
    return {"ratio": b / f, "forward_s": f, "backward_s": b, "workload": "single_puncture_64_dx0.25_50steps_ckpt10",
            "dJ_dlambda_gb": float(theta.grad[0]), "dJ_dg2": float(theta.grad[1]),
            "rhs_vjp_avg_ms": vjp_ms / max(vjp_n, 1), "rhs_vjps": vjp_n,
            "with_128_wide_stencil_column": wide,
            "reverse_pointwise_kernel": {"kernel": "k_vjp_point", "avg_launch_ms": pt_avg, "launches": pt_n,
                                         "executed_flops_per_cell": flops, "achieved": tflops, "peak": PEAK_FP64,
                                         "unit": "TFLOP/s", "frac": tflops / PEAK_FP64}}


def large_box(torch, G, I, steps=3):
    """256^3 two-puncture box, dx = M/16, lambda_gb = 0.2, g2 = 0.02: forward
    cell-updates/s of full RK4 steps (one warm-up step), and the pointwise
    kernel against its roofline as on the headline box."""
    n, dx = 256, 1.0 / 16.0
    p = I.default_params(lambda_gb=0.2, g2=0.02)
    u = torch.from_numpy(I.two_punctures(n, dx)).to("cuda")
    st = G.Stepper(G.make_params(p), G.box_of(u, dx, G.BC_FROZEN), u, 0.25 * dx)
    st.step()
    torch.cuda.synchronize()
    G.prof_begin(4 * steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        st.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    prof = G.prof_end()
    code, _ = st.status()
    del st, u
    torch.cuda.empty_cache()
    point_ms, point_n = prof["point"]
    fl = load_flops("full_theory")
    dom = roofline_point(fl["rk4_step"] / 4.0 - fl["stencils"], BYTES_STAGE, n ** 3, point_ms / max(point_n, 1))
    return {"workload": "two_punctures_256", "cells": n ** 3, "ms_per_step": ms,
            "cell_updates_per_s": n ** 3 / (ms * 1e-3), "steps": steps, "status": code,
            "dominant_kernel_roofline": {"kernel": "k_point_staged", "avg_launch_ms": dom["ms"],
                                         "achieved": dom["achieved"], "peak": dom["peak"], "unit": dom["unit"],
                                         "frac": dom["frac"]}}


def batched_speedup(torch, G, I, steps=4):
    """96 uneven boxes (levels 0-5): one-launch-per-box RK4 steps vs the batched
    form replayed from a hipGraph (one step per replay)."""
    spec = I.amr_boxes()
    states, dts = I.amr_states(spec)
    p = I.default_params()
    boxes = [G.make_box(b["dims"], b["dx"]) for b in spec]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        B = G.Batch(G.make_params(p), boxes, [torch.from_numpy(x).to("cuda") for x in states], dts)
        B.autotune(st)
        g = B.capture(st)

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                fn()
            e1.record(st)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        per_box = timed(lambda: B.step_perbox(st), steps)
        graph = timed(lambda: B.replay(g, st), steps)
        code, bits = B.status(st)
        chosen = [B.tile_variant(b) for b in range(len(spec))]
        # per-box launches again with every box on the tiled 16x8x4 stencil,
        # the per-box form's own best uniform choice on these boxes
        for b in range(len(spec)):
            B.set_tile_variant(b, 0)
        per_box_tiled = timed(lambda: B.step_perbox(st), steps)
        # and with every box on the stencil variant fastest for its own shape:
        # one RK4 step of a lone box of that shape timed with each variant a
        # batch box can take (grf_batch_set_tile_variant: 0..6 and 8)
        accepted = (0, 1, 2, 3, 4, 5, 6, 8)
        first = {}
        for b, bx in enumerate(spec):
            first.setdefault(tuple(bx["dims"]), b)
        v_single = G.get_tile_variant()
        best_v = {}
        for shp, b in first.items():
            S = G.Stepper(G.make_params(p), boxes[b], torch.from_numpy(states[b]).to("cuda"), dts[b])
            tv = {}
            for v in accepted:
                G.set_tile_variant(v)
                tv[v] = timed(lambda: S.step(st), 3)
            best_v[shp] = min(tv, key=tv.get)
        G.set_tile_variant(v_single)
        for b, bx in enumerate(spec):
            B.set_tile_variant(b, best_v[tuple(bx["dims"])])
        per_box_own = timed(lambda: B.step_perbox(st), steps)
        B.close()
    ncell = sum(int(b["dims"][0] * b["dims"][1] * b["dims"][2]) for b in spec)
    best_per_box = min(per_box, per_box_tiled, per_box_own)
    return {"per_box_ms_per_step": per_box, "per_box_tiled_ms_per_step": per_box_tiled,
            "per_box_own_variant_ms_per_step": per_box_own,
            "per_box_own_variants": sorted(set(best_v.values())),
            "batched_graph_ms_per_step": graph, "speedup": best_per_box / graph,
            "speedup_vs_same_variant_per_box": per_box / graph, "batched_cell_updates_per_s": ncell / (graph * 1e-3),
            "stencil_variants": sorted(set(chosen)), "cells": ncell, "boxes": len(spec), "status": code}


def other_rows(torch, G, I, params, box, u, st, n, dx, dt, ms_step, stream):
    """Timings of the diagnostics, the boundary rules, the decoupling limit and
    the sixth-order stencils on the headline box (each 5 calls after one warm-up)."""
    out = {}
    # constraint diagnostics (stencil stage + constraint kernel) on the same box
    G.constraints(G.make_params(params), box, st.u, st.ws)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        G.constraints(G.make_params(params), box, st.u, st.ws)
    c1.record(stream)
    torch.cuda.synchronize()
    out["constraints"] = {"ms_per_evaluation": c0.elapsed_time(c1) / 5,
                          "flops_per_cell": G.flops_per_cell(3)}
    c0.record(stream)
    for _ in range(5):
        G.energy_densities(G.make_params(params), box, st.u, st.ws)
    c1.record(stream)
    torch.cuda.synchronize()
    out["energy_densities"] = {"ms_per_evaluation": c0.elapsed_time(c1) / 5,
                               "flops_per_cell": G.flops_per_cell(4)}
    c0.record(stream)
    for _ in range(5):
        G.coupling_diagnostics(G.make_params(params), box, st.u, st.ws)
    c1.record(stream)
    torch.cuda.synchronize()
    out["coupling_diagnostics"] = {"ms_per_evaluation": c0.elapsed_time(c1) / 5,
                                   "flops_per_cell": G.flops_per_cell(6)}
    # per-face boundary rules: Sommerfeld on every face (ghosts integrated with
    # the radiative right-hand side) against the frozen-ghost step above
    origin = (-0.5 * n * dx + 0.5 * dx,) * 3
    flat = I.set_flat(I.empty_state((1, 1, 1)))[:, 3, 3, 3]
    bc = G.make_bc(["sommerfeld"] * 6, asymptote=flat)
    sb = G.StepperBC(G.make_params(params), G.box_of(u, dx, origin=origin), u.clone(), dt, bc)
    sb.step()
    torch.cuda.synchronize()
    c0.record(stream)
    for _ in range(5):
        sb.step()
    c1.record(stream)
    torch.cuda.synchronize()
    out["boundary_rules"] = {"ms_per_step_sommerfeld_faces": c0.elapsed_time(c1) / 5,
                             "ms_per_step_frozen": ms_step, "ghost_cells": G.bc_ghost_cells(box)}
    del sb
    # decoupling limit (scalar without backreaction) on the same box and path
    sd = G.Stepper(G.make_params(I.default_params(decoupled=1.0)), box, u.clone(), dt)
    sd.step()
    torch.cuda.synchronize()
    c0.record(stream)
    for _ in range(5):
        sd.step()
    c1.record(stream)
    torch.cuda.synchronize()
    out["decoupled"] = {"ms_per_step": c0.elapsed_time(c1) / 5, "ms_per_step_full_theory": ms_step,
                        "flops_per_cell": G.flops_per_cell(5)}
    del sd
    # sixth-order stencils on the same box (stencil kernel 32x8x32, staged pointwise kernel)
    s6 = G.Stepper(G.make_params(I.default_params(fd_order=6.0)), box, u.clone(), dt)
    s6.step()
    torch.cuda.synchronize()
    c0.record(stream)
    for _ in range(5):
        s6.step()
    c1.record(stream)
    torch.cuda.synchronize()
    ms6 = c0.elapsed_time(c1) / 5
    del s6
    # the sixth-order scheme on the same workload with four ghost layers
    # (sixth-order advection, eighth-difference dissipation)
    u4 = torch.from_numpy(I.single_puncture(n, dx, ng=4)).to(u.device)
    s4 = G.Stepper(G.make_params(I.default_params(fd_order=6.0)), G.box_of(u4, dx, G.BC_FROZEN, ng=4), u4, dt)
    s4.step()
    torch.cuda.synchronize()
    c0.record(stream)
    for _ in range(5):
        s4.step()
    c1.record(stream)
    torch.cuda.synchronize()
    out["sixth_order"] = {"ms_per_step": ms6, "ms_per_step_four_ghosts": c0.elapsed_time(c1) / 5,
                          "ms_per_step_fourth_order": ms_step}
    del s4, u4
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="box edge (cells)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the adjoint and batched measurements")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint/forward measurement (for kernel traces of the adjoint)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched vs per-box measurement (for kernel traces of the batch)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run one plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: libgrf has no multi-GPU path (the box-per-GPU "
              "sharding with halo exchange is a design, not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_06225_amd import grf as G
    from paper_2309_06225_amd import inputs as I

    if args.adjoint_only:
        print(json.dumps({"adjoint_forward_ratio": adjoint_ratio(torch, G, I)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_speedup(torch, G, I)}), flush=True)
        return

    n = args.n
    dx = 1.0 / 8.0
    dt = 0.25 * dx
    params = I.default_params()
    u_host = I.single_puncture(n, dx)
    u = torch.from_numpy(u_host).to("cuda")
    box = G.box_of(u, dx, G.BC_FROZEN)
    st = G.Stepper(G.make_params(params), box, u, dt)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        st.step()
    torch.cuda.synchronize()
    G.prof_begin(4 * args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        st.step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    prof = G.prof_end()
    code, bits = st.status()
    if code != 0:
        print(f"device status {code} bits {bits}", file=sys.stderr)
        sys.exit(1)

    ncell = n ** 3
    ms_step = ms_total / args.steps
    value = ncell * args.steps / (ms_total * 1e-3)
    point_ms, point_n = prof["point"]
    deriv_ms, deriv_n = prof["deriv"]
    avg_point = point_ms / max(point_n, 1)
    avg_stage = (point_ms + deriv_ms) / max(point_n, 1)
    # algorithmic flops per cell and stage from the oracle's op count: one RK4
    # step is four stages; the stencils and Kreiss-Oliger run in the stencil
    # kernel, the rest (algebra, Kreiss-Oliger weighting, stage update) in the
    # pointwise kernel, the dominant one
    fl = load_flops("full_theory_shift_advection" if params["shift_advec"] != 0.0 else "full_theory")
    stage_flops = fl["rk4_step"] / 4.0
    point_flops = stage_flops - fl["stencils"]
    kname = {0: "k_point", 2: "k_point_staged"}[G.get_stage_path()]
    dom = roofline_point(point_flops, BYTES_STAGE, ncell, avg_point)
    stage = roofline_point(stage_flops, BYTES_STAGE, ncell, avg_stage)
    traffic = load_traffic(kname, f"single_puncture_{n}")
    hbm_gbps = BYTES_STAGE * ncell / (avg_point * 1e-3) / 1e9
    # flops the generated kernel executes (its expression graph, common
    # subexpressions merged), for comparison with the algorithmic count
    exec_flops = G.flops_per_cell(1 if params["shift_advec"] != 0.0 else 0) + 27 * (1.0 + 13.0 / 4.0)
    roof = dict(dom)
    roof.update({"traffic": traffic,
                 "traffic_over_algorithmic": (traffic / (BYTES_STAGE * ncell)) if traffic else None,
                 "kernel": kname, "avg_launch_ms": avg_point, "launches": point_n,
                 "algorithmic_bytes_per_launch": BYTES_STAGE * ncell,
                 "flops_source": "oracle op count (profiles/flops_per_cell.json)",
                 "hbm_view": {"achieved": hbm_gbps, "peak": PEAK_HBM, "unit": "GB/s", "frac": hbm_gbps / PEAK_HBM},
                 "executed_flops_per_cell": exec_flops,
                 "executed_tflops": exec_flops * ncell / (avg_point * 1e-3) / 1e12,
                 "stage": stage})
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single_puncture_{n}", "cells": ncell, "ghosts": 3, "dx": dx, "dt": dt,
                   "bc": "frozen", "lambda_gb": params["lambda_gb"], "g2": params["g2"]},
        "roofline": roof,
        "kernels_ms_per_step": {"stencil": deriv_ms / args.steps, "pointwise_rk4": point_ms / args.steps},
        "rhs_cells_per_s": ncell * 4 * args.steps / (ms_total * 1e-3),
    }
    # measured peaks of this device beside the datasheet ones
    fp64_meas, copy_meas = G.measure_peaks()
    out["roofline"]["measured_peaks"] = {"fp64_tflops": fp64_meas, "copy_gbps": copy_meas,
                                         "frac_of_measured_fp64": dom["achieved"] / fp64_meas,
                                         "hbm_view_frac_of_measured_copy": hbm_gbps / copy_meas}
    if not args.no_extra:
        out.update(other_rows(torch, G, I, params, box, u, st, n, dx, dt, ms_step, stream))
        del st
        torch.cuda.empty_cache()
        out["adjoint_forward_ratio"] = adjoint_ratio(torch, G, I)
        out["batched"] = batched_speedup(torch, G, I)
        out["large_box"] = large_box(torch, G, I)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(params, u_host, dx, dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
