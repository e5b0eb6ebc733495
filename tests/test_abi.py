"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol,
and rejects bad arguments on the host without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "grf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2309_06225_amd import grf as G
    L = G.lib()
    names = declared_symbols()
    assert "grf_rhs_eval" in names and "grf_rk4_stage" in names and "grf_rhs_vjp" in names
    for n in names:
        assert hasattr(L, n), n


def test_host_side_validation_without_device():
    from paper_2309_06225_amd import grf as G
    L = G.lib()
    box = G.make_box((8, 8, 8), 0.25)
    assert L.grf_workspace_bytes(ctypes.byref(box)) >= 256 + 198 * 8 ** 3 * 8
    bad = G.make_box((8, 8, 8), 0.25)
    bad.ng = 2
    assert L.grf_workspace_bytes(ctypes.byref(bad)) == 0
    p = G.make_params()
    # null pointers are rejected before any HIP call
    code = L.grf_rhs_eval(ctypes.byref(p), ctypes.byref(box), None, None, None, 0, None)
    assert code != 0
    assert b"null" in L.grf_last_error() or b"workspace" in L.grf_last_error()
    assert L.grf_flops_per_cell(0) > 1000
    # four ghost layers: a valid shape, but only for the sixth-order scheme
    box4 = G.make_box((8, 8, 8), 0.25, ng=4)
    assert L.grf_workspace_bytes(ctypes.byref(box4)) == L.grf_workspace_bytes(ctypes.byref(box))
    assert L.grf_vjp_workspace_bytes(ctypes.byref(box4)) == L.grf_vjp_workspace_bytes(ctypes.byref(box))
    code = L.grf_rhs_eval(ctypes.byref(p), ctypes.byref(box4), None, None, None, 0, None)
    assert code == 7 and b"fd_order 6" in L.grf_last_error()
    bad.ng = 5
    assert L.grf_workspace_bytes(ctypes.byref(bad)) == 0
    short = G.make_box((8, 8, 8), 0.25, ng=4)
    short.field_stride = 14 ** 3
    assert L.grf_workspace_bytes(ctypes.byref(short)) == 0


def test_boundary_rules_rejected_on_the_host():
    """Invalid face rules are refused before any device work (the state pointer
    below is never dereferenced)."""
    from paper_2309_06225_amd import grf as G
    L = G.lib()
    box = G.make_box((8, 2, 8), 0.25, origin=(0.125, 0.125, 0.125))
    dummy = ctypes.c_void_p(8)
    cases = [
        G.make_bc(["periodic", "frozen"] + ["frozen"] * 4),                         # unpaired periodic face
        G.make_bc(["extrapolating"] * 6, extrap_order=2),                           # bad order
        G.make_bc(["frozen"] * 6, parity_phi=0),                                    # bad parity
        G.make_bc(["frozen", "frozen", "reflective", "frozen", "frozen", "frozen"]),  # 2 cells along y
    ]
    for bc in cases:
        assert L.grf_bc_fill(ctypes.byref(bc), ctypes.byref(box), dummy, None) == 1, L.grf_last_error()
    bad_rule = G.make_bc(["frozen"] * 6)
    bad_rule.rule[3] = 9
    assert L.grf_bc_fill(ctypes.byref(bad_rule), ctypes.byref(box), dummy, None) == 1
    # the radiative centre on a ghost cell centre (x index -1, y 0, z 3)
    som = G.make_bc(["sommerfeld"] * 6, centre=(0.125 - 0.25, 0.125, 0.125 + 3 * 0.25))
    assert L.grf_bc_ghost_rhs(ctypes.byref(som), ctypes.byref(box), dummy, ctypes.c_void_p(16), None) == 1
    assert b"centre" in L.grf_last_error()
    nan_speed = G.make_bc(["sommerfeld"] * 6, centre=(50.0, 0.0, 0.0), speed=[float("nan")] * 27)
    assert L.grf_bc_ghost_rhs(ctypes.byref(nan_speed), ctypes.byref(box), dummy, ctypes.c_void_p(16), None) == 1
    assert L.grf_bc_ghost_cells(ctypes.byref(box)) == 14 * 8 * 14 - 8 * 2 * 8


def test_static_stage_refuses_oversized_planes_on_the_host():
    """grf_rk4_stage_static checks a z-plane against its 128 MiB scratch before
    any device work (the pointers below are never dereferenced)."""
    from paper_2309_06225_amd import grf as G
    L = G.lib()
    p = G.make_params()
    box = G.make_box((300, 300, 4), 0.25)   # 90,000 cells per plane > 84,733
    ptr = [ctypes.c_void_p(8 * (k + 1)) for k in range(5)]
    code = L.grf_rk4_stage_static(ctypes.byref(p), ctypes.byref(box), 1, 0.1, ptr[0], ptr[1], ptr[2], ptr[3],
                                  ptr[4], None)
    assert code == 6 and b"static scratch" in L.grf_last_error()
    code = L.grf_rk4_stage_static(ctypes.byref(p), ctypes.byref(box), 1, 0.1, ptr[0], ptr[1], ptr[2], ptr[3],
                                  None, None)
    assert code == 1


def test_tile_variant_setting_on_the_host():
    """The single-box stencil variant: -1 (chosen per box, the default) or
    0..9; anything else is refused with GRF_EINVAL and leaves the setting."""
    from paper_2309_06225_amd import grf as G
    L = G.lib()
    v0 = L.grf_get_tile_variant()
    assert v0 == -1
    try:
        assert L.grf_set_tile_variant(9) == 0 and L.grf_get_tile_variant() == 9
        assert L.grf_set_tile_variant(10) == 1 and L.grf_get_tile_variant() == 9
        assert L.grf_set_tile_variant(-2) == 1 and L.grf_get_tile_variant() == 9
        assert L.grf_set_tile_variant(-1) == 0 and L.grf_get_tile_variant() == -1
    finally:
        L.grf_set_tile_variant(v0)
