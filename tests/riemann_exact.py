"""Exact solution of the 1D Riemann problem for the Euler equations of an
ideal gas (textbook construction: Toro, "Riemann Solvers and Numerical
Methods for Fluid Dynamics", ch. 4).  Used to pin the oracle's inviscid
limit on the Sod tube; it shares nothing with the oracle or the library.
"""
import numpy as np


def _f_side(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * np.sqrt(A / (p + B))
        df = np.sqrt(A / (B + p)) * (1.0 - (p - pk) / (2.0 * (B + p)))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _f_side(p, rl, pl, cl, g)
        fr, dfr = _f_side(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(1e-12, p - dp)
        if abs(p_new - p) < 1e-15 * p:
            p = p_new
            break
        p = p_new
    fl, _ = _f_side(p, rl, pl, cl, g)
    fr, _ = _f_side(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, g, xi):
    """(rho, u, p) at similarity coordinate xi = (x - x0) / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for i, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                rho[i], u[i], p[i] = (rl, ul, pl) if s < sl else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                head, tail = ul - cl, us - cs
                if s <= head:
                    rho[i], u[i], p[i] = rl, ul, pl
                elif s >= tail:
                    rho[i], u[i], p[i] = rs, us, ps
                else:
                    uu = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rho[i] = rl * (c / cl) ** (2.0 / (g - 1))
                    u[i] = uu
                    p[i] = pl * (c / cl) ** (2.0 * g / (g - 1))
        else:  # right of contact
            if ps > pr:  # right shock
                rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                rho[i], u[i], p[i] = (rs, us, ps) if s < sr else (rr, ur, pr)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / g)
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                head, tail = ur + cr, us + cs
                if s >= head:
                    rho[i], u[i], p[i] = rr, ur, pr
                elif s <= tail:
                    rho[i], u[i], p[i] = rs, us, ps
                else:
                    uu = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    rho[i] = rr * (c / cr) ** (2.0 / (g - 1))
                    u[i] = uu
                    p[i] = pr * (c / cr) ** (2.0 * g / (g - 1))
    return rho, u, p
