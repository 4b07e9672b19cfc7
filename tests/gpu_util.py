"""Shared helpers of the GPU tests (no step arithmetic here)."""
import numpy as np


def normwise(a, b):
    """Per-field max |a - b| / max |b| over all sub-grids and cells given
    arrays [count, F, ...]."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    for f in range(a.shape[1]):
        scale = np.max(np.abs(b[:, f]))
        out.append(np.max(np.abs(a[:, f] - b[:, f])) / (scale if scale > 0 else 1.0))
    return np.array(out)


def interior(U, n):
    return U[..., 3:3 + n, 3:3 + n, 3:3 + n]


def ghost_mask(n):
    M = n + 6
    m = np.ones((M, M, M), dtype=bool)
    m[3:3 + n, 3:3 + n, 3:3 + n] = False
    return m
