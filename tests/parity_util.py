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
