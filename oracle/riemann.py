"""Exact solution of the Riemann problem for an ideal gas (the Sod shock-tube
analytical solution the paper compares against in Sec. VI).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The star-region pressure p* is the root of
    F(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0,
where for side K with (rho_K, u_K, p_K) and sound speed c_K = sqrt(gamma p_K / rho_K)
    f_K(p) = (p - p_K) sqrt(A_K / (p + B_K))                 if p > p_K (shock)
           = 2 c_K / (gamma - 1) ((p / p_K)^((gamma-1)/(2 gamma)) - 1)   otherwise (rarefaction)
    A_K = 2 / ((gamma + 1) rho_K),  B_K = (gamma - 1) / (gamma + 1) p_K.
u* = (u_L + u_R + f_R(p*) - f_L(p*)) / 2.  The solution is self-similar in
x/t and sampled wave by wave.  F is monotone increasing in p, so a safeguarded
Newton iteration with a bisection bracket converges to the unique root.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, gamma):
    c = math.sqrt(gamma * pK / rho)
    if p > pK:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        s = math.sqrt(A / (p + B))
        return (p - pK) * s, s * (1.0 - 0.5 * (p - pK) / (p + B))
    e = (gamma - 1.0) / (2.0 * gamma)
    return (2.0 * c / (gamma - 1.0) * ((p / pK) ** e - 1.0),
            (1.0 / (rho * c)) * (p / pK) ** (-(gamma + 1.0) / (2.0 * gamma)))


def star_state(left, right, gamma):
    """(p*, u*, rho*_L, rho*_R) for left/right = (rho, u, p)."""
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    cL = math.sqrt(gamma * pL / rL)
    cR = math.sqrt(gamma * pR / rR)
    if 2.0 * (cL + cR) / (gamma - 1.0) <= uR - uL:
        raise ValueError("vacuum is generated; no star state")

    def F(p):
        a, da = _fK(p, rL, pL, gamma)
        b, db = _fK(p, rR, pR, gamma)
        return a + b + (uR - uL), da + db

    lo, hi = 1e-14, max(pL, pR)
    while F(hi)[0] < 0.0:
        hi *= 2.0
    p = 0.5 * (lo + hi)
    for _ in range(200):
        v, dv = F(p)
        if v > 0.0:
            hi = p
        else:
            lo = p
        pn = p - v / dv
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= 1e-15 * max(1.0, p):
            p = pn
            break
        p = pn
    fl = _fK(p, rL, pL, gamma)[0]
    fr = _fK(p, rR, pR, gamma)[0]
    u = 0.5 * (uL + uR) + 0.5 * (fr - fl)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    if p > pL:
        rsL = rL * ((p / pL) + g1) / (g1 * (p / pL) + 1.0)
    else:
        rsL = rL * (p / pL) ** (1.0 / gamma)
    if p > pR:
        rsR = rR * ((p / pR) + g1) / (g1 * (p / pR) + 1.0)
    else:
        rsR = rR * (p / pR) ** (1.0 / gamma)
    return p, u, rsL, rsR


def sample(left, right, gamma, s):
    """(rho, u, p) at similarity coordinates s = (x - x0) / t (array)."""
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    ps, us, rsL, rsR = star_state(left, right, gamma)
    cL = math.sqrt(gamma * pL / rL)
    cR = math.sqrt(gamma * pR / rR)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    for k, x in np.ndenumerate(s):
        if x <= us:  # left of the contact
            if ps > pL:  # left shock
                SL = uL - cL * math.sqrt((gamma + 1) / (2 * gamma) * ps / pL
                                         + (gamma - 1) / (2 * gamma))
                state = (rL, uL, pL) if x < SL else (rsL, us, ps)
            else:  # left rarefaction
                head = uL - cL
                tail = us - cL * (ps / pL) ** ((gamma - 1) / (2 * gamma))
                if x < head:
                    state = (rL, uL, pL)
                elif x > tail:
                    state = (rsL, us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cL + (gamma - 1) / 2 * (uL - x))
                    uu = 2.0 / (gamma + 1) * (cL + (gamma - 1) / 2 * uL + x)
                    rr = rL * (c / cL) ** (2 / (gamma - 1))
                    state = (rr, uu, pL * (c / cL) ** (2 * gamma / (gamma - 1)))
        else:  # right of the contact
            if ps > pR:  # right shock
                SR = uR + cR * math.sqrt((gamma + 1) / (2 * gamma) * ps / pR
                                         + (gamma - 1) / (2 * gamma))
                state = (rR, uR, pR) if x > SR else (rsR, us, ps)
            else:  # right rarefaction
                head = uR + cR
                tail = us + cR * (ps / pR) ** ((gamma - 1) / (2 * gamma))
                if x > head:
                    state = (rR, uR, pR)
                elif x < tail:
                    state = (rsR, us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cR - (gamma - 1) / 2 * (uR - x))
                    uu = 2.0 / (gamma + 1) * (-cR + (gamma - 1) / 2 * uR + x)
                    rr = rR * (c / cR) ** (2 / (gamma - 1))
                    state = (rr, uu, pR * (c / cR) ** (2 * gamma / (gamma - 1)))
        rho[k], u[k], p[k] = state
    return rho, u, p


def wave_speeds(left, right, gamma):
    """(slowest, fastest) signal speeds of the exact solution."""
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    ps, us, _, _ = star_state(left, right, gamma)
    cL = math.sqrt(gamma * pL / rL)
    cR = math.sqrt(gamma * pR / rR)
    if ps > pL:
        sl = uL - cL * math.sqrt((gamma + 1) / (2 * gamma) * ps / pL + (gamma - 1) / (2 * gamma))
    else:
        sl = uL - cL
    if ps > pR:
        sr = uR + cR * math.sqrt((gamma + 1) / (2 * gamma) * ps / pR + (gamma - 1) / (2 * gamma))
    else:
        sr = uR + cR
    return sl, sr
