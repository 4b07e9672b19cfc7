"""Exact solution of the 1-D Riemann problem for an ideal gas.

Written from the mathematics of the two-rarefaction / two-shock wave curves
(E. F. Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics",
3rd ed., Springer 2009, chapter 4): the star pressure p* is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot)
branch for p > p_K and the isentropic rarefaction branch otherwise.  It is
pinned by the published star state of Toro's Test 1 (tests/golden).
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rhoK, pK, cK, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rhoK)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        f = (p - pK) * s
        df = s * (1.0 - 0.5 * (p - pK) / (p + B))
    else:       # rarefaction
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * cK / (g - 1.0) * ((p / pK) ** e - 1.0)
        df = 1.0 / (rhoK * cK) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    """left/right = (rho, u, p).  Returns (p*, u*, rho*_L, rho*_R)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    du = uR - uL
    if 2.0 * (cL + cR) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated")
    p = max(1e-12, 0.5 * (pL + pR) - 0.125 * du * (rL + rR) * (cL + cR))
    for _ in range(200):
        fL, dL = _fK(p, rL, pL, cL, g)
        fR, dR = _fK(p, rR, pR, cR, g)
        pn = p - (fL + fR + du) / (dL + dR)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, cL, g)
    fR, _ = _fK(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)

    def rho_star(rK, pK):
        if p > pK:
            r = p / pK
            q = (g - 1.0) / (g + 1.0)
            return rK * (r + q) / (q * r + 1.0)
        return rK * (p / pK) ** (1.0 / g)

    return p, u, rho_star(rL, pL), rho_star(rR, pR)


def sample(left, right, g, xi):
    """Self-similar solution (rho, u, p) at xi = (x - x0)/t (array)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    ps, us, rsL, rsR = star_state(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for i, s in enumerate(xi.flat):
        if s <= us:  # left of the contact
            if ps > pL:  # left shock
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                w = (rL, uL, pL) if s <= SL else (rsL, us, ps)
            else:        # left rarefaction
                csL = cL * (ps / pL) ** ((g - 1) / (2 * g))
                head, tail = uL - cL, us - csL
                if s <= head:
                    w = (rL, uL, pL)
                elif s >= tail:
                    w = (rsL, us, ps)
                else:
                    uu = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s)
                    cc = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    rr = rL * (cc / cL) ** (2 / (g - 1))
                    w = (rr, uu, pL * (cc / cL) ** (2 * g / (g - 1)))
        else:        # right of the contact
            if ps > pR:  # right shock
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                w = (rR, uR, pR) if s >= SR else (rsR, us, ps)
            else:        # right rarefaction
                csR = cR * (ps / pR) ** ((g - 1) / (2 * g))
                head, tail = uR + cR, us + csR
                if s >= head:
                    w = (rR, uR, pR)
                elif s <= tail:
                    w = (rsR, us, ps)
                else:
                    uu = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s)
                    cc = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    rr = rR * (cc / cR) ** (2 / (g - 1))
                    w = (rr, uu, pR * (cc / cR) ** (2 * g / (g - 1)))
        rho.flat[i], u.flat[i], p.flat[i] = w
    return rho, u, p


def wave_positions(left, right, g):
    """(rarefaction head speed, shock speed) for a left-rarefaction /
    right-shock problem such as Sod's."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    ps, us, _, _ = star_state(left, right, g)
    SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
    return uL - cL, SR
