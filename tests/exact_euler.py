"""Exact Riemann solver of the 1D Euler equations (ideal gas).

Independent pin for the oracle's B = 0 limit: the textbook construction
(Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4):
the star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 with the shock /
rarefaction branches of f_K, found by Newton iteration; the solution is then
sampled along x/t.
"""
import math

import numpy as np


def _f_and_df(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = (p / pk) ** ((gamma - 1.0) / (2.0 * gamma))
    f = 2.0 * a / (gamma - 1.0) * (r - 1.0)
    df = 1.0 / (rho * a) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma, tol=1e-15):
    """(p*, u*, residual) for left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _f_and_df(p, rl, pl, gamma)
        fr, dfr = _f_and_df(p, rr, pr, gamma)
        g = fl + fr + (ur - ul)
        dp = g / (dfl + dfr)
        pn = max(p - dp, 1e-14)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, gamma)
    fr, _ = _f_and_df(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    res = fl + fr + (ur - ul)
    return p, u, res


def sample(left, right, gamma, xi):
    """(rho, u, p) arrays at similarity coordinates xi = (x - x0)/t."""
    ps, us, _ = star_state(left, right, gamma)
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    rho[n], u[n], p[n] = rl, ul, pl
                else:
                    rho[n] = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                    u[n], p[n] = us, ps
            else:  # left rarefaction
                shl = ul - al
                asl = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                stl = us - asl
                if s <= shl:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s >= stl:
                    rho[n] = rl * (ps / pl) ** (1.0 / gamma)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (gamma + 1) + g1 / al * (ul - s)
                    rho[n] = rl * c ** (2.0 / (gamma - 1))
                    u[n] = 2.0 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s)
                    p[n] = pl * c ** (2 * gamma / (gamma - 1))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    rho[n], u[n], p[n] = rr, ur, pr
                else:
                    rho[n] = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                    u[n], p[n] = us, ps
            else:  # right rarefaction
                shr = ur + ar
                asr = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                str_ = us + asr
                if s >= shr:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s <= str_:
                    rho[n] = rr * (ps / pr) ** (1.0 / gamma)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (gamma + 1) - g1 / ar * (ur - s)
                    rho[n] = rr * c ** (2.0 / (gamma - 1))
                    u[n] = 2.0 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s)
                    p[n] = pr * c ** (2 * gamma / (gamma - 1))
    return rho, u, p
