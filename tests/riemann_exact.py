"""Exact solution of the Riemann problem of the 1-D Euler equations (ideal
gas), a reference for the shock-capturing tests.

The star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 by Newton's method,
with f_K the velocity change across a shock (p > p_K, from the
Rankine-Hugoniot conditions) or across a rarefaction (p <= p_K, from the
isentropic relation and the Riemann invariant) connecting state K to the star
region; the solution is then sampled at x/t (Toro, Riemann Solvers and
Numerical Methods for Fluid Dynamics, ch. 4).
"""
import numpy as np


def _f(p, rho, pk, ck, g):
    """Velocity jump across the wave from a state (rho, pk, sound speed ck) to pressure p, and its derivative."""
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = np.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * ck)


def star_state(L, R, g=1.4):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    (rl, ul, pl), (rr, ur, pr) = L, R
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p = max(1e-12, p - dp)
        if abs(dp) < 1e-15 * p:
            break
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(L, R, s, g=1.4):
    """Primitive state (rho, u, p) at similarity coordinate s = x/t (arrays)."""
    (rl, ul, pl), (rr, ur, pr) = L, R
    ps, us = star_state(L, R, g)
    s = np.asarray(s, dtype=float)
    out = np.zeros((3,) + s.shape)
    gm, gp = (g - 1.0) / (g + 1.0), (g + 1.0)
    for side, (rk, uk, pk), sgn in ((0, L, -1.0), (1, R, 1.0)):
        ck = np.sqrt(g * pk / rk)
        # on this side of the contact: s < u* (left) or s >= u* (right)
        m = (s < us) if side == 0 else (s >= us)
        if ps > pk:   # shock
            S = uk + sgn * ck * np.sqrt((g + 1.0) / (2.0 * g) * ps / pk + (g - 1.0) / (2.0 * g))
            rs = rk * (ps / pk + gm) / (gm * ps / pk + 1.0)
            outer = m & ((s < S) if side == 0 else (s > S))
            inner = m & ~outer
            out[:, outer] = np.array([rk, uk, pk])[:, None]
            out[:, inner] = np.array([rs, us, ps])[:, None]
        else:         # rarefaction
            rs = rk * (ps / pk) ** (1.0 / g)
            cs = ck * (ps / pk) ** ((g - 1.0) / (2.0 * g))
            head, tail = uk + sgn * ck, us + sgn * cs
            outer = m & ((s < head) if side == 0 else (s > head))
            star = m & ((s > tail) if side == 0 else (s < tail))
            fan = m & ~outer & ~star
            out[:, outer] = np.array([rk, uk, pk])[:, None]
            out[:, star] = np.array([rs, us, ps])[:, None]
            sf = s[fan]
            u = 2.0 / gp * (-sgn * ck + (g - 1.0) / 2.0 * uk + sf)
            c = 2.0 / gp * ck - sgn * (g - 1.0) / gp * (uk - sf)
            out[0, fan] = rk * (c / ck) ** (2.0 / (g - 1.0))
            out[1, fan] = u
            out[2, fan] = pk * (c / ck) ** (2.0 * g / (g - 1.0))
    return out
