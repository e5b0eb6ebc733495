"""Seeded synthetic inputs for the 4dST/CCZ4 hot path.

This module is shared by the GPU path, the tests and the CPU oracle.  It holds
no arithmetic of the evolution method itself: only field names, parameter
values, coordinates and closed-form initial data (flat space with noise, a
puncture, a two-puncture superposition, scalar pulses), all evaluated on the
host with numpy.

State layout: float64 array of shape (27, nz + 6, ny + 6, nx + 6), field-major,
x fastest, with 3 ghost cells on every side.  Cell-centred coordinates,
x_i = x_lo + (i + 1/2) dx, with the box centred on ``centre``.
"""
from __future__ import annotations

import numpy as np

NG = 3
FIELDS = (
    "chi", "h11", "h12", "h13", "h22", "h23", "h33", "K",
    "A11", "A12", "A13", "A22", "A23", "A33", "Theta",
    "Gam1", "Gam2", "Gam3", "lapse", "shift1", "shift2", "shift3",
    "B1", "B2", "B3", "phi", "Pi",
)
NF = len(FIELDS)
IDX = {n: i for i, n in enumerate(FIELDS)}

# Parameter order of the flat 18-double parameter vector used by the oracle
# and by the GPU binding's marshalling.
PARAM_NAMES = (
    "lambda_gb", "g2", "a_gauge", "b_gauge", "kappa1", "kappa2", "kappa3",
    "lapse_coeff", "lapse_power", "lapse_advec",
    "shift_gamma_coeff", "shift_advec", "eta", "ko_sigma", "decoupled", "fd_order", "lambda_lin", "beta",
)


def default_params(**over) -> dict:
    """Couplings and gauge of the plain small workload: lambda(phi)=0.1 phi^2/4,
    g2=0.01, a=0.2, b=0.4, kappa=(0.1, 0, 1), 1+log lapse, Gamma-driver shift
    (B form, coefficient 3/4, eta=1, no shift advection), KO sigma=0.3."""
    p = dict(lambda_gb=0.1, g2=0.01, a_gauge=0.2, b_gauge=0.4,
             kappa1=0.1, kappa2=0.0, kappa3=1.0,
             lapse_coeff=2.0, lapse_power=1.0, lapse_advec=1.0,
             shift_gamma_coeff=0.75, shift_advec=0.0, eta=1.0, ko_sigma=0.3, decoupled=0.0, fd_order=4.0, lambda_lin=0.0,
             beta=0.0)
    for k, v in over.items():
        if k not in p:
            raise KeyError(k)
        p[k] = float(v)
    return p


def params_vector(p: dict) -> np.ndarray:
    return np.array([p[n] for n in PARAM_NAMES], dtype=np.float64)


def coords(dims, dx, centre=(0.0, 0.0, 0.0), ng=NG):
    """Cell-centre coordinate arrays (z, y, x order, including ng ghost layers)."""
    nx, ny, nz = dims
    axes = []
    for n, c in zip((nx, ny, nz), centre):
        i = np.arange(-ng, n + ng, dtype=np.float64)
        axes.append(c - 0.5 * n * dx + (i + 0.5) * dx)
    x, y, z = axes
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def empty_state(dims, ng=NG):
    nx, ny, nz = dims
    return np.zeros((NF, nz + 2 * ng, ny + 2 * ng, nx + 2 * ng), dtype=np.float64)


def set_flat(u):
    u[IDX["chi"]] = 1.0
    for n in ("h11", "h22", "h33"):
        u[IDX[n]] = 1.0
    u[IDX["lapse"]] = 1.0
    return u


def wrap_ghosts(u, ng=NG):
    """Periodic ghost fill of an input state (each ghost copies the interior cell
    congruent to it modulo the box size)."""
    inner = u[:, ng:-ng, ng:-ng, ng:-ng]
    return np.pad(inner, ((0, 0), (ng, ng), (ng, ng), (ng, ng)), mode="wrap")


def flat_noise_pulse(n=32, dx=0.25, seed=0, noise=1e-6, pulse=0.01, width2=4.0, ng=NG):
    """Periodic flat space + uniform noise on every field + Gaussian scalar pulse
    phi += pulse * exp(-r^2 / width2) (the interior does not depend on ng)."""
    dims = (n, n, n)
    u = set_flat(empty_state(dims, ng))
    rng = np.random.default_rng(seed)
    inner = (slice(ng, -ng),) * 3
    for f in range(NF):
        u[(f,) + inner] += rng.uniform(-noise, noise, size=(n, n, n))
    X, Y, Z = coords(dims, dx, ng=ng)
    r2 = X * X + Y * Y + Z * Z
    u[(IDX["phi"],) + inner] += pulse * np.exp(-r2[inner] / width2)
    return wrap_ghosts(u, ng)


def puncture(dims, dx, centre=(0.0, 0.0, 0.0), masses=((1.0, (0.0, 0.0, 0.0)),),
             phi_fn=None, ng=NG):
    """Conformally flat (superposed) puncture data, frozen ghosts included:
    chi^(-1/4) = 1 + sum_A m_A / (2 r_A) with r_A floored at dx/2; h = delta;
    A = K = Theta = Gamma = shift = B = 0; pre-collapsed lapse alpha = sqrt(chi);
    phi from phi_fn(X, Y, Z), Pi = 0."""
    u = empty_state(dims, ng)
    X, Y, Z = coords(dims, dx, centre, ng)
    psi = np.ones_like(X)
    for m, (cx, cy, cz) in masses:
        r = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2)
        r = np.maximum(r, 0.5 * dx)
        psi += m / (2.0 * r)
    chi = psi ** -4
    u[IDX["chi"]] = chi
    for n in ("h11", "h22", "h33"):
        u[IDX[n]] = 1.0
    u[IDX["lapse"]] = np.sqrt(chi)
    if phi_fn is not None:
        u[IDX["phi"]] = phi_fn(X, Y, Z)
    return u


def shell_pulse(amp=0.1, r0=4.0):
    def f(X, Y, Z):
        r = np.sqrt(X * X + Y * Y + Z * Z)
        return amp * np.exp(-(r - r0) ** 2)
    return f


def gaussian_pulse(amp=0.05, width2=25.0):
    def f(X, Y, Z):
        return amp * np.exp(-(X * X + Y * Y + Z * Z) / width2)
    return f


def single_puncture(n=128, dx=1.0 / 8.0, ng=NG):
    """One non-spinning puncture of mass 1 plus phi = 0.1 exp(-(r-4)^2)."""
    return puncture((n, n, n), dx, phi_fn=shell_pulse(), ng=ng)


def two_punctures(n=256, dx=1.0 / 16.0):
    """Masses 0.5 at (+-3, 0, 0) plus phi = 0.05 exp(-r^2/25)."""
    return puncture((n, n, n), dx, masses=((0.5, (3.0, 0.0, 0.0)), (0.5, (-3.0, 0.0, 0.0))),
                    phi_fn=gaussian_pulse())


def amr_boxes(nboxes=96, seed=2, edges=(16, 24, 32, 48, 64), levels=6, half=32.0):
    """Uneven boxes at refinement levels 0..levels-1 (dx = 2^-level), each placed
    uniformly at random so that it fits inside [-half, half]^3.  Returns a list of
    dicts with dims, dx, centre, level."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nboxes):
        dims = tuple(int(e) for e in rng.choice(edges, size=3))
        level = int(rng.integers(0, levels))
        dx = 2.0 ** (-level)
        centre = []
        for n in dims:
            hw = 0.5 * n * dx
            lo, hi = -half + hw, half - hw
            centre.append(float(rng.uniform(lo, hi)) if hi > lo else 0.0)
        out.append(dict(dims=dims, dx=dx, centre=tuple(centre), level=level))
    return out


def shell_mask(dims, dx, r_in=8.0, r_out=10.0, centre=(0.0, 0.0, 0.0)):
    """Interior cells with r_in < r < r_out (strict), as a bool array over the
    interior (nz, ny, nx)."""
    X, Y, Z = coords(dims, dx, centre)
    inner = (slice(NG, -NG),) * 3
    r = np.sqrt(X[inner] ** 2 + Y[inner] ** 2 + Z[inner] ** 2)
    return (r > r_in) & (r < r_out)


def interior(u, ng=NG):
    return u[..., ng:-ng, ng:-ng, ng:-ng]


def amr_states(boxes):
    """The single-puncture data (mass 1 at the origin, phi = 0.1 exp(-(r-4)^2))
    sampled at the cells of each box; returns (states, dts) with dt = dx/4."""
    states, dts = [], []
    for bx in boxes:
        states.append(puncture(bx["dims"], bx["dx"], centre=bx["centre"], phi_fn=shell_pulse()))
        dts.append(0.25 * bx["dx"])
    return states, dts
