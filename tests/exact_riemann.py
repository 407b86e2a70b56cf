"""Exact solution of the 1D Euler Riemann problem for an ideal gas.

Test infrastructure: the textbook construction (pressure function of the
star region solved by Newton's method, then sampling of the self-similar
wave pattern) as given in Toro, "Riemann Solvers and Numerical Methods for
Fluid Dynamics", ch. 4.  Used to pin the whole scheme on the Sod problem.
"""
import math

import numpy as np


def _fK(p, rho, pK, cK, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (p + B))
    r = p / pK  # rarefaction
    f = 2.0 * cK / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * cK) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g=1.4):
    rL, uL, pL = L
    rR, uR, pR = R
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    p = max(1e-10, 0.5 * (pL + pR) - 0.125 * (uR - uL) * (rL + rR) * (cL + cR))
    for _ in range(100):
        fL, dL = _fK(p, rL, pL, cL, g)
        fR, dR = _fK(p, rR, pR, cR, g)
        dp = (fL + fR + uR - uL) / (dL + dR)
        pn = max(1e-12, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, cL, g)
    fR, _ = _fK(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def sample(L, R, S, g=1.4):
    """Primitive state (rho, u, p) at similarity coordinate S = x/t."""
    rL, uL, pL = L
    rR, uR, pR = R
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    ps, us = star_state(L, R, g)
    gm = (g - 1.0) / (g + 1.0)
    if S <= us:  # left of contact
        if ps > pL:
            SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
            if S <= SL:
                return rL, uL, pL
            return rL * (ps / pL + gm) / (gm * ps / pL + 1.0), us, ps
        SHL = uL - cL
        cs = cL * (ps / pL) ** ((g - 1) / (2 * g))
        STL = us - cs
        if S <= SHL:
            return rL, uL, pL
        if S >= STL:
            return rL * (ps / pL) ** (1 / g), us, ps
        u = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + S)
        c = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - S))
        rho = rL * (c / cL) ** (2 / (g - 1))
        return rho, u, pL * (c / cL) ** (2 * g / (g - 1))
    if ps > pR:
        SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
        if S >= SR:
            return rR, uR, pR
        return rR * (ps / pR + gm) / (gm * ps / pR + 1.0), us, ps
    SHR = uR + cR
    cs = cR * (ps / pR) ** ((g - 1) / (2 * g))
    STR = us + cs
    if S >= SHR:
        return rR, uR, pR
    if S <= STR:
        return rR * (ps / pR) ** (1 / g), us, ps
    u = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + S)
    c = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - S))
    rho = rR * (c / cR) ** (2 / (g - 1))
    return rho, u, pR * (c / cR) ** (2 * g / (g - 1))


def zone_average_density(L, R, n, t, x0=0.5, g=1.4, sub=64):
    """Zone averages of the exact density on [0,1] with n zones at time t."""
    h = 1.0 / n
    out = np.empty(n)
    for i in range(n):
        xs = (i + (np.arange(sub) + 0.5) / sub) * h
        out[i] = np.mean([sample(L, R, (x - x0) / t, g)[0] for x in xs])
    return out
