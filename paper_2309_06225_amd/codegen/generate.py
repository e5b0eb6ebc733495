"""Emit the generated device code of the pointwise algebra.

Writes, next to the hand-written kernels:
  gen_layout.h    component layout of the derivative buffer and flop counts
  gen_rhs.inc     forward right-hand side (two variants: with/without shift advection)
  gen_vjp.inc     its vector-Jacobian product
The include files expect the including kernel to define the access macros
GRF_U(f), GRF_D(c), GRF_P(name), GRF_RHS(f, v), GRF_PIVCHK(v), and for the VJP
GRF_W(f), GRF_BAR_U(f, v), GRF_BAR_D(c, v), GRF_BAR_TH(q, v).
"""
from __future__ import annotations

import os
import sys

from . import ccz4_4dst as M
from .expr import count_flops, emit, emit_staged, vjp

NCOMP_D1 = 3 * len(M.D1_FIELDS)
NCOMP_D2 = 6 * len(M.D2_FIELDS)
OFF_D1, OFF_D2 = 0, NCOMP_D1
OFF_ADV = NCOMP_D1 + NCOMP_D2
OFF_KO = OFF_ADV + M.NF
NCOMP = OFF_KO + M.NF


def comp_of(name: str) -> int:
    if name.startswith("d1_"):
        _, f, k = name.split("_")
        return OFF_D1 + 3 * M.D1_FIELDS.index(int(f)) + int(k)
    if name.startswith("d2_"):
        _, f, q = name.split("_")
        return OFF_D2 + 6 * M.D2_FIELDS.index(int(f)) + int(q)
    if name.startswith("adv"):
        return OFF_ADV + int(name[3:])
    raise KeyError(name)


def input_expr(name: str) -> str:
    if name.startswith("u"):
        return f"GRF_U({int(name[1:])})"
    return f"GRF_D({comp_of(name)})"


def param_expr(name: str) -> str:
    return f"GRF_P({name})"


def forward_code(shift_advec: bool):
    b = M.build(shift_advec)
    g = b["graph"]
    # outputs that do not need the per-cell solve first, then the pivot checks
    # (which pull in the solve), then the rest
    from .expr import reachable
    solve_nodes = reachable(b["pivots"])
    rhs = b["rhs"]
    indep = [f for f in range(M.NF) if not (reachable([rhs[f]]) & {p.idx for p in b["pivots"]})]
    dep = [f for f in range(M.NF) if f not in indep]
    outs = [rhs[f] for f in indep] + b["pivot_check"] + [rhs[f] for f in dep]
    names = ([f"GRF_RHS({f}, {{}})" for f in indep] + ["GRF_PIVCHK({})"] * len(b["pivot_check"])
             + [f"GRF_RHS({f}, {{}})" for f in dep])
    del solve_nodes
    code = emit(g, outs, names, input_expr, param_expr, order="dfs")
    flops, ops = count_flops(g, b["rhs"])
    return code, flops, ops


# staged item slots per buffer of the staged pointwise kernel (64 lanes x 8 bytes
# each; two buffers per wave)
STAGE_SLOTS = 40


def _stage_key(name: str):
    if name.startswith("u"):
        return ("U", int(name[1:]))
    return ("D", comp_of(name))


def forward_code_staged(shift_advec: bool, rhs_only: bool, decoupled: bool = False, general_coupling: bool = True):
    """Forward right-hand side with staged inputs (see emit_staged).  Each
    right-hand-side statement also stages its Kreiss-Oliger component and, for
    the RK4 stage modes, u0 and the accumulator of its field.  decoupled: the
    decoupling limit (its constant pivot entries are not checked)."""
    b = M.build(shift_advec, decoupled, general_coupling)
    g = b["graph"]
    from .expr import reachable
    rhs = b["rhs"]
    pivots = [p for p in b["pivots"] if p.op != "c"] if decoupled else b["pivots"]
    checks = [p for p in b["pivot_check"] if p.op != "c"] if decoupled else b["pivot_check"]
    indep = [f for f in range(M.NF) if not (reachable([rhs[f]]) & {p.idx for p in pivots})]
    dep = [f for f in range(M.NF) if f not in indep]
    outs = [rhs[f] for f in indep] + checks + [rhs[f] for f in dep]

    def rhs_stmt(f):
        if rhs_only:
            return (f"GRF_RHS_ST({f}, {{v}}, {{b}}, {{s0}}, 0, 0)", [("KO", f)])
        return (f"GRF_RHS_ST({f}, {{v}}, {{b}}, {{s0}}, {{s1}}, {{s2}})", [("KO", f), ("U0", f), ("ACC", f)])

    stmts = ([rhs_stmt(f) for f in indep] + [("GRF_PIVCHK({v})", [])] * len(checks)
             + [rhs_stmt(f) for f in dep])
    # greedy list schedule keeping few values live (ties in heavier-operand-first
    # order): a fifth less spilling in this kernel than that order alone
    return emit_staged(g, outs, stmts, _stage_key, param_expr, STAGE_SLOTS, order="greedy")


def constraints_code(decoupled: bool = False):
    """Hamiltonian and momentum constraints of one cell: GRF_CON(q, v), q = 0
    Hamiltonian, 1..3 momentum (they do not involve the advection sums); in
    the decoupling limit without the scalar's sources."""
    b = M.build(False, decoupled=decoupled)
    g = b["graph"]
    outs = b["constraints"]
    names = [f"GRF_CON({q}, {{}})" for q in range(len(outs))]
    code = emit(g, outs, names, input_expr, param_expr, order="dfs")
    flops, ops = count_flops(g, outs)
    return code, flops


def energy_code():
    """Energy densities of the canonical, X^2 and Gauss-Bonnet terms of one
    cell: GRF_CON(q, v), q = 0, 1, 2."""
    b = M.build(False)
    g = b["graph"]
    outs = M.energies(b)
    names = [f"GRF_CON({q}, {{}})" for q in range(len(outs))]
    code = emit(g, outs, names, input_expr, param_expr, order="dfs")
    flops, ops = count_flops(g, outs)
    return code, flops


def coupling_code():
    """Gauss-Bonnet invariant, the weak-coupling indicators and the
    determinant of the per-cell system of one cell: GRF_CON(q, v), q = 0..3."""
    b = M.build(False)
    g = b["graph"]
    outs = M.coupling(b)
    names = [f"GRF_CON({q}, {{}})" for q in range(len(outs))]
    code = emit(g, outs, names, input_expr, param_expr, order="dfs")
    flops, ops = count_flops(g, outs)
    return code, flops


def _quad_flops(shift_advec: bool):
    """Flops of the default code: the quadratic coupling alone."""
    b = M.build(shift_advec, general_coupling=False)
    return count_flops(b["graph"], b["rhs"])[0]


def _dec_flops():
    b = M.build(False, decoupled=True)
    return count_flops(b["graph"], b["rhs"])[0]


def vjp_code(shift_advec: bool, decoupled: bool = False):
    """Reverse of the pointwise algebra with the quadratic coupling alone (the
    adjoint takes gradients with respect to lambda_gb and g2; the general
    coupling's nodes would only lengthen the tape)."""
    b = M.build(shift_advec, decoupled=decoupled, general_coupling=False)
    g = b["graph"]
    w = [g.input(f"w{f}") for f in range(M.NF)]
    leaves = [n for n in g.nodes if n.op == "in" and not n.name.startswith("w")]
    wrt = leaves + b["theta"]
    bars = vjp(g, b["rhs"], w, wrt)
    outs, names = [], []
    zero_u, zero_d = [], []
    for leaf, bar in zip(wrt, bars):
        if leaf.op == "p":
            name = f"GRF_BAR_TH({0 if leaf.name == 'lambda_gb' else 1}, {{}})"
        elif leaf.name.startswith("u"):
            name = f"GRF_BAR_U({int(leaf.name[1:])}, {{}})"
        else:
            name = f"GRF_BAR_D({comp_of(leaf.name)}, {{}})"
        if bar.op == "c" and bar.val == 0.0:
            # every cotangent slot is written, zeros included
            (zero_u if leaf.op == "in" and leaf.name.startswith("u") else zero_d).append(name.format("0.0"))
            continue
        outs.append(bar)
        names.append(name)

    def inexpr(name):
        if name.startswith("w"):
            return f"GRF_W({int(name[1:])})"
        return input_expr(name)

    code = emit(g, outs, names, inexpr, param_expr)
    code = "\n".join("  " + z + ";" for z in zero_u + zero_d) + "\n" + code
    flops, ops = count_flops(g, outs)
    return code, flops, ops


# every block of generated code rounds exactly as written: explicit fma() where
# the fusion plan says so, no contraction by the compiler
PRAGMA = "#pragma clang fp contract(off)\n"


def block(cond: str, then_code: str, else_code: str) -> str:
    return (f"if constexpr ({cond}) {{\n" + PRAGMA + then_code + "\n} else {\n" + PRAGMA + else_code + "\n}\n")


def main(outdir: str):
    os.makedirs(outdir, exist_ok=True)
    fw0, fl0, ops0 = forward_code(False)
    fw1, fl1, ops1 = forward_code(True)
    vj0, vfl0, vops0 = vjp_code(False)
    vj1, vfl1, vops1 = vjp_code(True)
    hdr = [
        "// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.",
        "#pragma once",
        f"#define GRF_NCOMP {NCOMP}        // components per cell in the derivative buffer",
        f"#define GRF_OFF_D1 {OFF_D1}",
        f"#define GRF_OFF_D2 {OFF_D2}",
        f"#define GRF_OFF_ADV {OFF_ADV}",
        f"#define GRF_OFF_KO {OFF_KO}",
        f"#define GRF_FLOPS_RHS {_quad_flops(False)}     // graph flops per cell, no shift advection",
        f"#define GRF_FLOPS_RHS_SHIFTADV {_quad_flops(True)}",
        "// with the general coupling (linear and exponential terms of lambda(phi))",
        f"#define GRF_FLOPS_RHS_GENERAL {fl0}",
        f"#define GRF_FLOPS_VJP {vfl0}",
        f"#define GRF_FLOPS_VJP_SHIFTADV {vfl1}",
        f"#define GRF_FLOPS_CONSTRAINTS {constraints_code()[1]}",
        f"#define GRF_FLOPS_ENERGY {energy_code()[1]}",
        f"#define GRF_FLOPS_COUPLING {coupling_code()[1]}",
        f"#define GRF_FLOPS_RHS_DECOUPLED {_dec_flops()}",
        f"#define GRF_STAGE_SLOTS {STAGE_SLOTS}  // slots per buffer of the staged pointwise kernel",
        "// parameters read by the generated code (derived combinations precomputed on the host)",
        "struct grf_point_params {",
    ] + [f"  double {n};" for n in M.PARAMS] + [
        "};",
        "// d1 component of (field f, axis k): GRF_OFF_D1 + 3*d1_slot[f] + k (-1: not stored)",
        "static constexpr int grf_d1_slot[27] = {" + ",".join(
            str(M.D1_FIELDS.index(f)) if f in M.D1_FIELDS else "-1" for f in range(M.NF)) + "};",
        "// d2 component of (field f, packed xx,xy,xz,yy,yz,zz q): GRF_OFF_D2 + 6*d2_slot[f] + q",
        "static constexpr int grf_d2_slot[27] = {" + ",".join(
            str(M.D2_FIELDS.index(f)) if f in M.D2_FIELDS else "-1" for f in range(M.NF)) + "};",
        "// 1 where the stencil stage adds the field's advection sum into the field's",
        "// Kreiss-Oliger slot instead of storing it (index: shift advection off / on)",
        "static constexpr int grf_adv_merged[2][27] = {" + ", ".join(
            "{" + ",".join("1" if f in M.merged_adv(sa) else "0" for f in range(M.NF)) + "}" for sa in (False, True))
        + "};",
        "// field of each d1 / d2 slot (inverse of the tables above)",
        f"static constexpr int grf_d1_field[{len(M.D1_FIELDS)}] = {{" + ",".join(str(f) for f in M.D1_FIELDS) + "};",
        f"static constexpr int grf_d2_field[{len(M.D2_FIELDS)}] = {{" + ",".join(str(f) for f in M.D2_FIELDS) + "};",
    ]
    with open(os.path.join(outdir, "gen_layout.h"), "w") as fh:
        fh.write("\n".join(hdr) + "\n")
    with open(os.path.join(outdir, "gen_rhs.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// forward right-hand side: {fl0} flops/cell ({ops0})\n")
        fh.write(block("GRF_SHIFT_ADVEC", fw1, fw0))
    # the default staged kernel: the quadratic coupling alone (without the
    # general coupling's nodes the schedule keeps its measured spill count);
    # the general coupling has its own staged variant below
    staged = {}
    for ro in (True, False):
        for sa in (True, False):
            staged[(ro, sa)] = forward_code_staged(sa, ro, general_coupling=False)
    with open(os.path.join(outdir, "gen_rhs_staged.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// forward right-hand side with inputs staged through two buffers of {STAGE_SLOTS} slots;\n")
        fh.write("// phases (rhs only / stage, shift advection on / off): "
                 + ", ".join(f"{v[1]}" for v in staged.values()) + "\n")
        fh.write("if constexpr (GRF_STAGE_RHS_ONLY) {\n")
        fh.write(block("GRF_SHIFT_ADVEC", staged[(True, True)][0], staged[(True, False)][0]))
        fh.write("} else {\n")
        fh.write(block("GRF_SHIFT_ADVEC", staged[(False, True)][0], staged[(False, False)][0]))
        fh.write("}\n")
    staged_lin = {}
    for ro in (True, False):
        for sa in (True, False):
            staged_lin[(ro, sa)] = forward_code_staged(sa, ro, general_coupling=True)
    with open(os.path.join(outdir, "gen_rhs_staged_lin.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write("// with the general coupling (linear and exponential terms), staged as gen_rhs_staged.inc;\n")
        fh.write("// phases (rhs only / stage, shift advection on / off): "
                 + ", ".join(f"{v[1]}" for v in staged_lin.values()) + "\n")
        fh.write("if constexpr (GRF_STAGE_RHS_ONLY) {\n")
        fh.write(block("GRF_SHIFT_ADVEC", staged_lin[(True, True)][0], staged_lin[(True, False)][0]))
        fh.write("} else {\n")
        fh.write(block("GRF_SHIFT_ADVEC", staged_lin[(False, True)][0], staged_lin[(False, False)][0]))
        fh.write("}\n")
    staged_dec = {}
    for ro in (True, False):
        for sa in (True, False):
            staged_dec[(ro, sa)] = forward_code_staged(sa, ro, decoupled=True)
    with open(os.path.join(outdir, "gen_rhs_staged_dec.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write("// decoupling limit (the scalar does not source the metric), staged as gen_rhs_staged.inc;\n")
        fh.write("// phases (rhs only / stage, shift advection on / off): "
                 + ", ".join(f"{v[1]}" for v in staged_dec.values()) + "\n")
        fh.write("if constexpr (GRF_STAGE_RHS_ONLY) {\n")
        fh.write(block("GRF_SHIFT_ADVEC", staged_dec[(True, True)][0], staged_dec[(True, False)][0]))
        fh.write("} else {\n")
        fh.write(block("GRF_SHIFT_ADVEC", staged_dec[(False, True)][0], staged_dec[(False, False)][0]))
        fh.write("}\n")
    con, cfl = constraints_code()
    with open(os.path.join(outdir, "gen_constraints.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// Hamiltonian and momentum constraints: {cfl} flops/cell\n")
        fh.write("{\n" + PRAGMA + con + "\n}\n")
    cond, cdfl = constraints_code(decoupled=True)
    with open(os.path.join(outdir, "gen_constraints_dec.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// Hamiltonian and momentum constraints in the decoupling limit: {cdfl} flops/cell\n")
        fh.write("{\n" + PRAGMA + cond + "\n}\n")
    en, efl = energy_code()
    with open(os.path.join(outdir, "gen_energy.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// energy densities of the canonical, X^2 and Gauss-Bonnet terms: {efl} flops/cell\n")
        fh.write("{\n" + PRAGMA + en + "\n}\n")
    cp, cpfl = coupling_code()
    with open(os.path.join(outdir, "gen_coupling.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// Gauss-Bonnet invariant, weak-coupling indicators, system determinant: {cpfl} flops/cell\n")
        fh.write("{\n" + PRAGMA + cp + "\n}\n")
    with open(os.path.join(outdir, "gen_vjp.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// vector-Jacobian product: {vfl0} flops/cell ({vops0})\n")
        fh.write(block("GRF_SHIFT_ADVEC", vj1, vj0))
    vd0, vdfl0, vdops0 = vjp_code(False, decoupled=True)
    vd1, _, _ = vjp_code(True, decoupled=True)
    with open(os.path.join(outdir, "gen_vjp_dec.inc"), "w") as fh:
        fh.write("// Generated by paper_2309_06225_amd/codegen/generate.py -- do not edit.\n")
        fh.write(f"// vector-Jacobian product in the decoupling limit: {vdfl0} flops/cell ({vdops0})\n")
        fh.write(block("GRF_SHIFT_ADVEC", vd1, vd0))
    return dict(flops_rhs=fl0, flops_rhs_shiftadv=fl1, flops_vjp=vfl0, ops=ops0, vops=vops0)


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.dirname(__file__)), "csrc", "gen")
    print(main(out))
