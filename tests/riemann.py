"""Exact solution of the Riemann problem for an ideal gas (test helper).

Textbook method (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4): Newton iteration on the pressure function for the star
pressure, then sampling of the self-similar solution. Independent of the
oracle; used to pin its shock capturing on the Sod problem.
"""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - pk) / (2.0 * (B + p)))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g=1.4):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-12)
        if abs(pn - p) < 1e-14 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(x, t, x0, left, right, g=1.4):
    """Density, velocity and pressure at positions x (array) and time t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, len(x)))
    for k, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                SL = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= SL:
                    out[:, k] = (rl, ul, pl)
                else:
                    out[:, k] = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                SHL, STL = ul - cl, us - csl
                if s <= SHL:
                    out[:, k] = (rl, ul, pl)
                elif s > STL:
                    out[:, k] = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    r = rl * (c / cl) ** (2.0 / (g - 1))
                    out[:, k] = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                SR = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= SR:
                    out[:, k] = (rr, ur, pr)
                else:
                    out[:, k] = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                SHR, STR = ur + cr, us + csr
                if s >= SHR:
                    out[:, k] = (rr, ur, pr)
                elif s < STR:
                    out[:, k] = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    r = rr * (c / cr) ** (2.0 / (g - 1))
                    out[:, k] = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out


def right_shock_speed(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    ps, _ = star_state(rl, ul, pl, rr, ur, pr, g)
    cr = math.sqrt(g * pr / rr)
    return ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
