"""TEST INFRASTRUCTURE -- exact Riemann solver of the 1-D gamma-law Euler
equations (the textbook construction: Toro, "Riemann Solvers and Numerical
Methods for Fluid Dynamics", ch. 4).  Used by the tests to pin the two-shock
solver (O6) and the whole step on a shock tube.

The star pressure p* solves f_L(p) + f_R(p) + (u_R - u_L) = 0 with
  f_K(p) = (p - p_K) sqrt(A_K / (p + B_K))                  p > p_K (shock)
  f_K(p) = 2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1)   p <= p_K (rarefaction)
  A_K = 2 / ((gamma+1) rho_K),  B_K = (gamma-1)/(gamma+1) p_K,
and u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.
"""
import math


def _f(p, rho, pk, g):
    c = math.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * c / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * c)


def star(L, R, g, tol=1e-15, maxit=200):
    """Star pressure and velocity for left/right primitive states (rho, u, p)."""
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    p = max(0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr), 1e-8 * min(pl, pr))
    for _ in range(maxit):
        fl, dfl = _f(p, rl, pl, g)
        fr, dfr = _f(p, rr, pr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        if pn <= 0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, g)
    fr, _ = _f(p, rr, pr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(L, R, g, s):
    """Exact solution (rho, u, p) at similarity coordinate s = x/t."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star(L, R, g)
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:  # left of the contact
        cl = math.sqrt(g * pl / rl)
        if ps > pl:
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if s <= sl:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
        shl = ul - cl
        if s <= shl:
            return rl, ul, pl
        csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if s >= us - csl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
        rho = rl * (c / cl) ** (2.0 / (g - 1.0))
        return rho, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    cr = math.sqrt(g * pr / rr)
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if s >= sr:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
    shr = ur + cr
    if s >= shr:
        return rr, ur, pr
    csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if s <= us + csr:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
    rho = rr * (c / cr) ** (2.0 / (g - 1.0))
    return rho, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def shock_speeds(L, R, g):
    """(left wave speed, right wave speed) of the shocks, None for a rarefaction."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, _ = star(L, R, g)
    left = right = None
    if ps > pl:
        cl = math.sqrt(g * pl / rl)
        left = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
    if ps > pr:
        cr = math.sqrt(g * pr / rr)
        right = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
    return left, right
