"""Exact solution of the 1-D Riemann problem for the Euler equations of an ideal
gas (test helper; textbook construction, e.g. Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4): the star pressure solves
f_L(p) + f_R(p) + (u_R - u_L) = 0 with f_K the shock (Rankine-Hugoniot) or
rarefaction (isentropic) relation of side K; the solution is self-similar in
x / t."""
import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = np.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    e = (g - 1.0) / (2.0 * g)     # rarefaction
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * ck)


def star_state(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(xi, left, right, g=1.4):
    """(rho, u, p) at x/t = xi (array) for the left/right primitive states."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for side, (rk, uk, pk, ck, sgn) in (("L", (rl, ul, pl, cl, -1.0)), ("R", (rr, ur, pr, cr, 1.0))):
        msk = xi < us if side == "L" else xi >= us
        x = xi[msk]
        if ps > pk:  # shock
            rs = rk * (ps / pk + gm) / (gm * ps / pk + 1.0)
            S = uk + sgn * ck * np.sqrt((g + 1.0) / (2.0 * g) * ps / pk + (g - 1.0) / (2.0 * g))
            out = (x < S) if side == "L" else (x > S)
            r_, u_, p_ = np.where(out, rk, rs), np.where(out, uk, us), np.where(out, pk, ps)
        else:  # rarefaction
            rs = rk * (ps / pk) ** (1.0 / g)
            cs = ck * (ps / pk) ** ((g - 1.0) / (2.0 * g))
            head, tail = uk + sgn * ck, us + sgn * cs
            outside = (x < head) if side == "L" else (x > head)
            star = (x > tail) if side == "L" else (x < tail)
            # inside the fan
            uf = 2.0 / (g + 1.0) * (-sgn * ck + (g - 1.0) / 2.0 * uk + x)
            cf = -sgn * (uf - x)
            rf = rk * (cf / ck) ** (2.0 / (g - 1.0))
            pf = pk * (cf / ck) ** (2.0 * g / (g - 1.0))
            r_ = np.where(outside, rk, np.where(star, rs, rf))
            u_ = np.where(outside, uk, np.where(star, us, uf))
            p_ = np.where(outside, pk, np.where(star, ps, pf))
        rho[msk], u[msk], p[msk] = r_, u_, p_
    return rho, u, p
