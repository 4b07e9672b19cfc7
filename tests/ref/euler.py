"""Textbook ideal-gas Euler relations, written independently of the oracle,
for closed-form checks: conserved state and physical flux of a primitive
state (rho, vx, vy, vz, p, passive...)."""
from __future__ import annotations

import numpy as np

GAMMA = 5.0 / 3.0


def cons(W, g=GAMMA):
    W = np.asarray(W, dtype=np.float64)
    rho, vx, vy, vz, p = W[0], W[1], W[2], W[3], W[4]
    out = [rho, rho * vx, rho * vy, rho * vz,
           p / (g - 1.0) + 0.5 * rho * (vx ** 2 + vy ** 2 + vz ** 2)]
    out += [W[k] for k in range(5, W.shape[0])]
    return np.array(out)


def flux(W, d, g=GAMMA):
    """Flux of mass, momentum, total energy and passive densities through a
    face normal to axis d."""
    W = np.asarray(W, dtype=np.float64)
    U = cons(W, g)
    v = W[1 + d]
    p = W[4]
    F = U * v
    F[1 + d] += p
    F[4] += p * v
    return F


def sound_speed(W, g=GAMMA):
    return np.sqrt(g * W[4] / W[0])
