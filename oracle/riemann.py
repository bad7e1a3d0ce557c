"""Exact solution of the 1-D Riemann problem for a polytropic ideal gas.

Test infrastructure (part of the oracle package).  The shock-tube pins compare
the PonD solution with the exact Euler solution; this is the textbook exact
solver: the star pressure is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0,
where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the isentropic
rarefaction branch for p <= p_K, found by Newton iteration; the solution is
then sampled along rays x/t.  The paper's shock-capturing claims (Sec.
"Numerical applications", the high-Mach jet) rely on recovering the Euler
limit; its adiabatic exponent is gamma = (c_v + r)/c_v (Eq. spec_heat).
"""
from __future__ import annotations

import math

import numpy as np


def _branch(p, rho_k, p_k, c_k, g):
    """f_K(p) and its derivative for side K."""
    if p > p_k:                                   # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        return (p - p_k) * s, s * (1.0 - 0.5 * (p - p_k) / (B + p))
    r = p / p_k                                   # rarefaction
    f = 2.0 * c_k / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho_k * c_k) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, gamma):
    """(p*, u*) for left = (rho, u, p), right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated; not handled")
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dl = _branch(p, rl, pl, cl, g)
        fr, dr = _branch(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _branch(p, rl, pl, cl, g)
    fr, _ = _branch(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, gamma, xi):
    """Exact (rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, gamma)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s <= us:                                # left of the contact
            if ps > pl:
                S = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s < S:
                    rho[n], u[n], p[n] = rl, ul, pl
                else:
                    rho[n] = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                    u[n], p[n] = us, ps
            else:
                head = ul - cl
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                tail = us - cs
                if s < head:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s > tail:
                    rho[n] = rl * (ps / pl) ** (1.0 / g)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * (ul - s))
                    u[n] = 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * ul + s)
                    rho[n] = rl * (c / cl) ** (2.0 / (g - 1))
                    p[n] = pl * (c / cl) ** (2.0 * g / (g - 1))
        else:                                      # right of the contact
            if ps > pr:
                S = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s > S:
                    rho[n], u[n], p[n] = rr, ur, pr
                else:
                    rho[n] = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                    u[n], p[n] = us, ps
            else:
                head = ur + cr
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                tail = us + cs
                if s > head:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s < tail:
                    rho[n] = rr * (ps / pr) ** (1.0 / g)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (g + 1) * (cr - 0.5 * (g - 1) * (ur - s))
                    u[n] = 2.0 / (g + 1) * (-cr + 0.5 * (g - 1) * ur + s)
                    rho[n] = rr * (c / cr) ** (2.0 / (g - 1))
                    p[n] = pr * (c / cr) ** (2.0 * g / (g - 1))
    return rho, u, p


def wave_speeds(left, right, gamma):
    """dict of the wave speeds: left/right shock speed or rarefaction head/tail, contact."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, gamma)
    out = {"contact": us, "p_star": ps, "u_star": us}
    if ps > pl:
        out["left_shock"] = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
    else:
        out["left_head"] = ul - cl
        out["left_tail"] = us - cl * (ps / pl) ** ((g - 1) / (2 * g))
    if ps > pr:
        out["right_shock"] = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
    else:
        out["right_head"] = ur + cr
        out["right_tail"] = us + cr * (ps / pr) ** ((g - 1) / (2 * g))
    return out
