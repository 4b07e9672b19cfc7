"""Shared helpers of the GPU tests (no step arithmetic here)."""
import os

import numpy as np


def normwise(a, b):
    """Per-field max |a - b| / max |b| over all sub-grids and cells given
    arrays [count, F, ...] (the pooled metric)."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    for f in range(a.shape[1]):
        scale = np.max(np.abs(b[:, f]))
        out.append(np.max(np.abs(a[:, f] - b[:, f])) / (scale if scale > 0 else 1.0))
    return np.array(out)


def normwise_each(a, b):
    """Per sub-grid and per field: max |a - b| / max |b| over that sub-grid's
    cells, an array [count, F].  A sub-grid's field that is zero everywhere
    in b must be zero in a too (its entry is then max |a|).  Unlike the
    pooled metric this sees errors in sub-grids whose values are far below
    the batch maximum (e.g. the 1e-10 atmosphere of a polytrope)."""
    a = np.asarray(a)
    b = np.asarray(b)
    count, nf = a.shape[0], a.shape[1]
    d = np.abs(a - b).reshape(count, nf, -1).max(axis=2)
    s = np.abs(b).reshape(count, nf, -1).max(axis=2)
    return np.where(s > 0, d / np.where(s > 0, s, 1.0), d)


def interior(U, n):
    return U[..., 3:3 + n, 3:3 + n, 3:3 + n]


def ghost_mask(n):
    M = n + 6
    m = np.ones((M, M, M), dtype=bool)
    m[3:3 + n, 3:3 + n, 3:3 + n] = False
    return m


def oracle_threads():
    """Threads for the oracle in GPU tests: the host's cores, at most 16."""
    return max(1, min(os.cpu_count() or 1, 16))
