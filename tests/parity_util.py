"""Helpers for GPU-vs-oracle comparisons."""
import numpy as np

NG = 3


def rel_err_per_field(g, o, interior=True, ng=NG):
    """e_f = max |g - o| / max |o| per field (over interior cells); a field whose
    oracle values are all zero is scaled by the largest field maximum instead."""
    if interior:
        s = (slice(None),) + (slice(ng, -ng),) * 3
        g, o = g[s], o[s]
    g = g.reshape(g.shape[0], -1)
    o = o.reshape(o.shape[0], -1)
    num = np.abs(g - o).max(axis=1)
    den = np.abs(o).max(axis=1)
    glob = den.max() if den.max() > 0 else 1.0
    den = np.where(den > 0, den, glob)
    return num / den


def no_exchange_pivots(A):
    """Pivots of Gaussian elimination without row exchanges."""
    M = np.array(A, dtype=float)
    n = len(M)
    piv = np.empty(n)
    for k in range(n):
        piv[k] = M[k, k]
        for i in range(k + 1, n):
            M[i, k:] -= M[i, k] / M[k, k] * M[k, k:]
    return piv


def exchange_state():
    """A point state (u[27], d1[27, 3], d2[27, 6]) and a coupling lambda_GB
    (g2 = 0.1) at which the per-cell system has a zero in its first diagonal
    entry yet is well conditioned: lambda_GB is bisected, with the oracle's
    assembled matrix, to the zero crossing of A[0][0] along a scan (seeded
    random state near flat space)."""
    from oracle import oracle as O
    from paper_2309_06225_amd import inputs as I
    idx = I.IDX
    rng = np.random.default_rng(11)
    u = np.zeros(27)
    u[idx["chi"]] = 1.0 + 0.3 * rng.random()
    for n in ("h11", "h22", "h33"):
        u[idx[n]] = 1.0
    for n in ("h12", "h13", "h23"):
        u[idx[n]] = 0.1 * rng.standard_normal()
    u[idx["lapse"]] = 1.0
    for n in ("A11", "A12", "A13", "A22", "A23", "A33"):
        u[idx[n]] = 0.5 * rng.standard_normal()
    for n in ("K", "phi", "Pi"):
        u[idx[n]] = rng.standard_normal()
    d1 = 0.5 * rng.standard_normal((27, 3))
    d2 = 0.5 * rng.standard_normal((27, 6))

    def a00(lg):
        p = I.default_params(lambda_gb=lg, g2=0.1)
        return O.rhs_point(I.params_vector(p), u, d1, d2, np.zeros((27, 3)))[1]["A"][0, 0]

    lgs = np.geomspace(0.05, 5.0, 60)
    vals = [a00(lg) for lg in lgs]
    k = next(k for k in range(1, len(lgs)) if np.sign(vals[k]) != np.sign(vals[k - 1]))
    a, b, sa = lgs[k - 1], lgs[k], np.sign(vals[k - 1])
    for _ in range(80):
        m = 0.5 * (a + b)
        if np.sign(a00(m)) == sa:
            a = m
        else:
            b = m
    return u, d1, d2, a


def quadratic_box(u, d1, d2, dims, dx, ng=NG):
    """State (27, nz + 2 ng, ny + 2 ng, nx + 2 ng) whose every field is the
    quadratic u + d1 . x + x^T H x / 2 about the box's central cell (ghosts
    included), H from the packed second derivatives (xx, xy, xz, yy, yz, zz);
    fourth-order centred and upwinded differences reproduce d1 and d2 there."""
    nx, ny, nz = dims
    c = [(n - 1) // 2 + ng for n in dims]
    x = (np.arange(nx + 2 * ng) - c[0]) * dx
    y = (np.arange(ny + 2 * ng) - c[1]) * dx
    z = (np.arange(nz + 2 * ng) - c[2]) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    out = np.empty((27,) + Z.shape)
    for f in range(27):
        xx, xy, xz, yy, yz, zz = d2[f]
        out[f] = (u[f] + d1[f, 0] * X + d1[f, 1] * Y + d1[f, 2] * Z
                  + 0.5 * (xx * X * X + yy * Y * Y + zz * Z * Z) + xy * X * Y + xz * X * Z + yz * Y * Z)
    return out


def oracle_region_rk4(oracle, pv, u, dx, dt, nsteps, r0, w, ng=NG):
    """The oracle's state after nsteps RK4 steps with frozen ghosts, on the
    interior cells r0[a] .. r0[a] + w - 1 along each axis (x, y, z) of the
    ghost-inclusive state u, computed on a sub-box cut from u.

    A cell's value after n steps depends only on cells within 3 (4n - 1) of it:
    the first stage reads the initial state, and each of the 4n - 1 later stages
    reads at most three cells further.  So a sub-box that reaches that far
    beyond the region inside the box (and to the box's own ghosts where the
    region is closer to a face: those are frozen in both runs) gives the region
    the whole box's values.  Returns the region, shape (27, w, w, w)."""
    m = 3 * (4 * nsteps - 1)
    n = [u.shape[3] - 2 * ng, u.shape[2] - 2 * ng, u.shape[1] - 2 * ng]
    lo = [max(0, r0[a] - m) for a in range(3)]
    hi = [min(n[a], r0[a] + w + m) for a in range(3)]
    sub = np.ascontiguousarray(u[:, lo[2]:hi[2] + 2 * ng, lo[1]:hi[1] + 2 * ng, lo[0]:hi[0] + 2 * ng])
    o, flags = oracle.rk4(pv, sub, dx, dt, nsteps, periodic=False)
    assert flags == 0, flags
    s = [r0[a] - lo[a] + ng for a in range(3)]
    return o[:, s[2]:s[2] + w, s[1]:s[1] + w, s[0]:s[0] + w]
