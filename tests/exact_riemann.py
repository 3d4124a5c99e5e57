"""Exact solution of the Riemann problem for the 1-D Euler equations of an
ideal gas, written from the mathematics of the problem (independent of the
oracle): the star pressure is the root of the pressure function

    f(p) = f_L(p) + f_R(p) + (u_R - u_L),

with f_K the shock (Rankine-Hugoniot) branch for p > p_K and the rarefaction
(isentropic Riemann invariant) branch otherwise; the root is found by Newton
iteration from the two-rarefaction guess, then the self-similar solution is
sampled at x/t.  Used to pin the oracle on shock tubes (Sec. 4.1 of the paper
and the colliding-states case its text mentions).
"""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        f = (p - pk) * s
        df = s * (1.0 - 0.5 * (p - pk) / (B + p))
    else:
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0)
        df = (1.0 / (rho * ck)) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(WL, WR, g):
    rL, uL, pL = WL
    rR, uR, pR = WR
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    e = (g - 1.0) / (2.0 * g)
    # two-rarefaction initial guess
    p = ((cL + cR - 0.5 * (g - 1.0) * (uR - uL)) / (cL / pL ** e + cR / pR ** e)) ** (1.0 / e)
    p = max(p, 1e-12)
    for _ in range(100):
        fL, dL = _fk(p, rL, pL, cL, g)
        fR, dR = _fk(p, rR, pR, cR, g)
        f = fL + fR + (uR - uL)
        pn = p - f / (dL + dR)
        if pn <= 0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fk(p, rL, pL, cL, g)
    fR, _ = _fk(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def sample(WL, WR, g, xi):
    """Solution (rho, u, p) at similarity coordinate xi = (x - x0) / t."""
    rL, uL, pL = WL
    rR, uR, pR = WR
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    ps, us = star_state(WL, WR, g)
    gp = (g + 1.0) / (2.0 * g)
    gm = (g - 1.0) / (2.0 * g)
    if xi <= us:  # left of the contact
        if ps > pL:  # left shock
            SL = uL - cL * math.sqrt(gp * ps / pL + gm)
            if xi <= SL:
                return rL, uL, pL
            r = rL * ((ps / pL + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pL + 1.0))
            return r, us, ps
        # left rarefaction
        csL = cL * (ps / pL) ** gm
        SHL, STL = uL - cL, us - csL
        if xi <= SHL:
            return rL, uL, pL
        if xi >= STL:
            return rL * (ps / pL) ** (1.0 / g), us, ps
        c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * (uL - xi))
        u = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * uL + xi)
        r = rL * (c / cL) ** (2.0 / (g - 1.0))
        return r, u, pL * (c / cL) ** (2.0 * g / (g - 1.0))
    # right of the contact
    if ps > pR:
        SR = uR + cR * math.sqrt(gp * ps / pR + gm)
        if xi >= SR:
            return rR, uR, pR
        r = rR * ((ps / pR + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pR + 1.0))
        return r, us, ps
    csR = cR * (ps / pR) ** gm
    SHR, STR = uR + cR, us + csR
    if xi >= SHR:
        return rR, uR, pR
    if xi <= STR:
        return rR * (ps / pR) ** (1.0 / g), us, ps
    c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * (uR - xi))
    u = 2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * uR + xi)
    r = rR * (c / cR) ** (2.0 / (g - 1.0))
    return r, u, pR * (c / cR) ** (2.0 * g / (g - 1.0))


def profile(WL, WR, g, x, x0, t):
    out = np.array([sample(WL, WR, g, (xx - x0) / t) for xx in x])
    return out[:, 0], out[:, 1], out[:, 2]
