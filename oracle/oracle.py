"""ctypes wrapper of the plain C++ CPU oracle (``grf_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark load this module; the GPU library never does, and this module
imports nothing from the GPU package.

States are numpy float64 arrays of shape (27, nz+6, ny+6, nx+6).  Parameters
are the 18-double vector (lambda_gb, g2, a, b, kappa1, kappa2, kappa3,
lapse_coeff, lapse_power, lapse_advec, shift_gamma_coeff, shift_advec, eta,
ko_sigma, decoupled, fd_order, lambda_lin, beta).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grf_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
NF = 27
NG = 3

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_rhs.argtypes = [_dp, _ip, _dp, _dp, _dp]
        L.oracle_rhs_cells.argtypes = [_dp, _ip, _dp, _dp, ctypes.c_int, _ip, _dp]
        L.oracle_rhs_cs.argtypes = [_dp, _dp, _ip, _dp, _dp, _dp, _dp, _dp]
        L.oracle_constraints.argtypes = [_dp, _ip, _dp, _dp, _dp, _dp]
        L.oracle_energy_densities.argtypes = [_dp, _ip, _dp, _dp, _dp]
        L.oracle_coupling.argtypes = [_dp, _ip, _dp, _dp, _dp]
        L.oracle_fill_periodic.argtypes = [_ip, _dp]
        L.oracle_fill_bc.argtypes = [_ip, _dp, _dp, _dp]
        L.oracle_ghost_rhs.argtypes = [_ip, _dp, _dp, _dp, _dp]
        L.oracle_rk4_bc.argtypes = [_dp, _ip, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp]
        L.oracle_rk4.argtypes = [_dp, _ip, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
        L.oracle_rk4_ld.argtypes = [_dp, _ip, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
        L.oracle_rk4_cs.argtypes = [_dp, _dp, _ip, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.oracle_rhs_point.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_enforce.argtypes = [_ip, _dp, ctypes.c_double, ctypes.c_double]
        L.oracle_gepp.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_gepp.restype = ctypes.c_double
        L.oracle_stencils.argtypes = [_ip, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_flops_per_cell.argtypes = [_dp, _ip, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _dims(u, ng=NG):
    """nx, ny, nz and the ghost count, as the oracle's box reads them."""
    nz, ny, nx = (s - 2 * ng for s in u.shape[1:])
    return np.array([nx, ny, nz, ng], dtype=np.int32)


def _spacing(dx):
    if np.isscalar(dx):
        dx = (dx, dx, dx)
    return np.array(dx, dtype=np.float64)


def rhs(params, u, dx, ng=NG):
    """Right-hand side (incl. Kreiss-Oliger) on interior cells; ghosts of the result are 0.
    ng: ghost layers of u (4 only with the sixth-order scheme)."""
    u = _c(u)
    out = np.zeros_like(u)
    p = _c(params)
    dims = _dims(u, ng)
    flags = lib().oracle_rhs(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u), _d(out))
    return out, flags


def rhs_cells(params, u, dx, cells, ng=NG):
    """Right-hand side at interior cells given as an (n, 3) array of (i, j, k)."""
    u = _c(u)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    out = np.zeros((cells.shape[0], NF))
    p = _c(params)
    dims = _dims(u, ng)
    flags = lib().oracle_rhs_cells(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u), cells.shape[0],
                                   cells.ctypes.data_as(_ip), _d(out))
    return out, flags


def rhs_cs(params, theta_im, u_re, u_im, dx, ng=NG):
    """Complex-step right-hand side. Returns (real part, imaginary part)."""
    u_re = _c(u_re)
    u_im = _c(u_im) if u_im is not None else np.zeros_like(u_re)
    r_re = np.zeros_like(u_re)
    r_im = np.zeros_like(u_re)
    p = _c(params)
    ti = _c(theta_im)
    dims = _dims(u_re, ng)
    lib().oracle_rhs_cs(_d(p), _d(ti), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u_re), _d(u_im),
                        _d(r_re), _d(r_im))
    return r_re, r_im


def constraints(params, u, dx, ng=NG):
    """Hamiltonian (nz,ny,nx) and momentum (3,nz,ny,nx) constraints on the interior."""
    u = _c(u)
    ham = np.zeros(u.shape[1:])
    mom = np.zeros((NF,) + u.shape[1:])  # only the first 3 fields are written
    p = _c(params)
    dims = _dims(u, ng)
    lib().oracle_constraints(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u), _d(ham), _d(mom))
    s = (slice(ng, -ng),) * 3
    return ham[s], mom[(slice(0, 3),) + s]


def energy_densities(params, u, dx, ng=NG):
    """Energy densities (3,nz,ny,nx) of the canonical, X^2 and Gauss-Bonnet
    terms of the action on the interior."""
    u = _c(u)
    rho = np.zeros((NF,) + u.shape[1:])  # only the first 3 fields are written
    p = _c(params)
    dims = _dims(u, ng)
    lib().oracle_energy_densities(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u), _d(rho))
    s = (slice(ng, -ng),) * 3
    return rho[(slice(0, 3),) + s]


FACE_RULES = {"frozen": 0, "periodic": 1, "reflective": 2, "extrapolating": 3, "sommerfeld": 4}


def pack_bc(bc):
    """Boundary rules as the oracle reads them.  bc: dict with `rules` (six of
    FACE_RULES' names, faces x-, x+, y-, y+, z-, z+), `extrap_order`, `origin`
    (coordinates of interior cell (0,0,0)), `centre`, `speed[27]`,
    `asymptote[27]`, `parity_phi`."""
    v = [float(FACE_RULES[r]) for r in bc["rules"]] + [float(bc.get("extrap_order", 1))]
    v += [float(x) for x in bc.get("origin", (0.0, 0.0, 0.0))] + [float(x) for x in bc.get("centre", (0.0, 0.0, 0.0))]
    v += [float(x) for x in bc.get("speed", np.ones(NF))] + [float(x) for x in bc.get("asymptote", np.zeros(NF))]
    v += [float(bc.get("parity_phi", 1))]
    assert len(v) == 68
    return np.array(v)


def coupling(params, u, dx, ng=NG):
    """(4,nz,ny,nx) on the interior: the Gauss-Bonnet invariant, the
    weak-coupling indicators |lambda'(phi)| sqrt|L_GB| and |2 g2 X|, and the
    determinant of the per-cell system."""
    u = _c(u)
    out = np.zeros((NF,) + u.shape[1:])  # only the first 4 fields are written
    p = _c(params)
    dims = _dims(u, ng)
    lib().oracle_coupling(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u), _d(out))
    s = (slice(ng, -ng),) * 3
    return out[(slice(0, 4),) + s]


def fill_bc(u, dx, bc, ng=NG):
    """Ghosts of periodic, reflective and extrapolating faces refilled (new state)."""
    u = _c(u).copy()
    dims = _dims(u, ng)
    lib().oracle_fill_bc(dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(pack_bc(bc)), _d(u))
    return u


def ghost_rhs(u, dx, bc, ng=NG):
    """Right-hand side in the ghost cells (radiative on Sommerfeld faces, 0 on
    the others); interior cells are 0."""
    u = _c(u)
    r = np.zeros_like(u)
    dims = _dims(u, ng)
    lib().oracle_ghost_rhs(dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(pack_bc(bc)), _d(u), _d(r))
    return r


def rk4_bc(params, u, dx, dt, nsteps, bc, ng=NG):
    """nsteps classic RK4 steps with per-face boundary rules; (state, flags)."""
    u = _c(u).copy()
    p = _c(params)
    dims = _dims(u, ng)
    flags = lib().oracle_rk4_bc(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(pack_bc(bc)), float(dt),
                                int(nsteps), _d(u))
    return u, flags


def fill_periodic(u, ng=NG):
    u = _c(u).copy()
    dims = _dims(u, ng)
    lib().oracle_fill_periodic(dims.ctypes.data_as(_ip), _d(u))
    return u


def rk4(params, u, dx, dt, nsteps, periodic, ng=NG):
    """nsteps classic RK4 steps; returns (new state, flags)."""
    u = _c(u).copy()
    p = _c(params)
    dims = _dims(u, ng)
    flags = lib().oracle_rk4(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), 1 if periodic else 0,
                             float(dt), int(nsteps), _d(u))
    return u, flags


def rk4_ld(params, u, dx, dt, nsteps, periodic, ng=NG):
    """nsteps classic RK4 steps carried out in long double (x87 extended
    precision) throughout, the result rounded to double: a reference for the
    double-precision results; returns (new state, flags)."""
    u = _c(u).copy()
    p = _c(params)
    dims = _dims(u, ng)
    flags = lib().oracle_rk4_ld(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), 1 if periodic else 0,
                                float(dt), int(nsteps), _d(u))
    return u, flags


def rk4_cs(params, theta_im, u_re, u_im, dx, dt, nsteps, periodic, ng=NG):
    """Complex-step RK4: returns (real state, imaginary state)."""
    u_re = _c(u_re).copy()
    u_im = _c(u_im).copy()
    p = _c(params)
    ti = _c(theta_im)
    dims = _dims(u_re, ng)
    lib().oracle_rk4_cs(_d(p), _d(ti), dims.ctypes.data_as(_ip), _d(_spacing(dx)), 1 if periodic else 0,
                        float(dt), int(nsteps), _d(u_re), _d(u_im))
    return u_re, u_im


def rhs_point(params, u, d1, d2, adv):
    """Pointwise right-hand side from values u[27], d1[27,3], d2[27,6], adv[27,3].
    Returns (rhs[27], extra dict, flags)."""
    p = _c(params)
    u = _c(u)
    d1 = _c(d1)
    d2 = _c(d2)
    adv = _c(adv)
    out = np.zeros(NF)
    extra = np.zeros(75)
    flags = lib().oracle_rhs_point(_d(p), _d(u), _d(d1), _d(d2), _d(adv), _d(out), _d(extra))
    ex = dict(ham=extra[0], mom=extra[1:4], C=extra[4:10], p=extra[10],
              A=extra[11:60].reshape(7, 7), b=extra[60:67], pivot_ratio=extra[67], rho=extra[68:71],
              lgb=extra[71], weak=extra[72:74], detA=extra[74])
    return out, ex, flags


def enforce(u, chi_min, lapse_min, ng=NG):
    """Post-stage enforcement on the interior cells (returns a new state)."""
    u = _c(u).copy()
    dims = _dims(u, ng)
    lib().oracle_enforce(dims.ctypes.data_as(_ip), _d(u), float(chi_min), float(lapse_min))
    return u


def gepp(A, b):
    A = _c(A)
    b = _c(b)
    x = np.zeros(b.shape[0])
    ratio = lib().oracle_gepp(int(b.shape[0]), _d(A), _d(b), _d(x))
    return x, ratio


def stencils(f, dx, i, j, k, order=4, ng=NG):
    """Stencils (centred order 4 or 6) of a scalar field f (shape (nz+2ng, ny+2ng, nx+2ng))
    at interior cell (i,j,k): dict with d1[3], d2[6], adv_plus[3], adv_minus[3], ko."""
    f = _c(f)
    nz, ny, nx = (s - 2 * ng for s in f.shape)
    dims = np.array([nx, ny, nz, ng], dtype=np.int32)
    out = np.zeros(16)
    lib().oracle_stencils(dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(f), i, j, k, int(order), _d(out))
    return dict(d1=out[0:3], d2=out[3:9], adv_plus=out[9:12], adv_minus=out[12:15], ko=out[15])


def flops_per_cell(params, u, dx, ng=NG):
    """Algorithmic flops per interior cell counted on the oracle's own code
    (add, sub, mul, div, sqrt, cbrt, exp, pow 1 each; constants folded; only
    operations the outputs depend on): dict with `rhs` (one right-hand side,
    Kreiss-Oliger included), `stencils` (its stencil and Kreiss-Oliger part)
    and `rk4_step` (one RK4 step, four right-hand sides and the updates, the
    box taken as periodic).  u: a small box of generic (non-degenerate) data."""
    u = _c(u)
    out = np.zeros(3)
    p = _c(params)
    dims = _dims(u, ng)
    lib().oracle_flops_per_cell(_d(p), dims.ctypes.data_as(_ip), _d(_spacing(dx)), _d(u), _d(out))
    return dict(rhs=out[0], stencils=out[1], rk4_step=out[2])
