"""Exact Riemann solver for the 1D Euler equations of a gamma-law gas.

Textbook construction (two-rarefaction / two-shock pressure function, Newton
iteration for the star pressure, self-similar sampling), used as the
epsilon -> 0 limit of the kinetic scheme: gamma = 3 for d_v = 1
(E = rho T / 2 + rho u^2 / 2, p = rho T) and gamma = 2 for d_v = 2
(E = p + rho |u|^2 / 2).
"""
import math

import numpy as np


def _fK(p, rho, pK, gamma):
    c = math.sqrt(gamma * pK / rho)
    if p > pK:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pK) / (B + p))
    else:
        f = 2.0 * c / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * c) * (p / pK) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(L, R, gamma):
    rl, ul, pl = L
    rr, ur, pr = R
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _fK(p, rl, pl, gamma)
        fr, dfr = _fK(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, gamma)
    fr, _ = _fK(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, gamma, xi):
    """(rho, u, p) at the similarity coordinate(s) xi = (x - x0) / t."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star_state(L, R, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = np.zeros((len(np.atleast_1d(xi)), 3))
    for n, s in enumerate(np.atleast_1d(xi)):
        if s <= us:   # left of contact
            cl = math.sqrt(gamma * pl / rl)
            if ps > pl:   # left shock
                sl = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    out[n] = (rl, ul, pl)
                else:
                    out[n] = (rl * (ps / pl + g1) / (g1 * ps / pl + 1.0), us, ps)
            else:         # left rarefaction
                cs = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                if s <= ul - cl:
                    out[n] = (rl, ul, pl)
                elif s >= us - cs:
                    out[n] = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    u = 2.0 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + s)
                    c = 2.0 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                    rho = rl * (c / cl) ** (2.0 / (gamma - 1))
                    out[n] = (rho, u, pl * (c / cl) ** (2.0 * gamma / (gamma - 1)))
        else:         # right of contact
            cr = math.sqrt(gamma * pr / rr)
            if ps > pr:   # right shock
                sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    out[n] = (rr, ur, pr)
                else:
                    out[n] = (rr * (ps / pr + g1) / (g1 * ps / pr + 1.0), us, ps)
            else:         # right rarefaction
                cs = cr * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                if s >= ur + cr:
                    out[n] = (rr, ur, pr)
                elif s <= us + cs:
                    out[n] = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    u = 2.0 / (gamma + 1) * (-cr + (gamma - 1) / 2 * ur + s)
                    c = 2.0 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                    rho = rr * (c / cr) ** (2.0 / (gamma - 1))
                    out[n] = (rho, u, pr * (c / cr) ** (2.0 * gamma / (gamma - 1)))
    return out
