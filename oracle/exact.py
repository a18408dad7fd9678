"""Closed-form and exact solutions of the Euler equations used to pin the oracle
(test infrastructure only).

* piston-driven shock: a piston pushed at constant speed into gas at rest (the set-up of
  the paper's open-ended shock-tube test, Sec. 3.5);
* stationary normal shock (Rankine-Hugoniot; the paper's stationary-shock tests, Sec. 3.2
  and 3.3);
* the exact solution of the 1D Riemann problem for a perfect gas (pressure-function root
  by Newton iteration, then sampling of the self-similar fan), written from the jump
  and isentrope relations.
"""
import math

import numpy as np


def sound_speed(gamma, rho, p):
    return math.sqrt(gamma * p / rho)


def piston_shock(gamma, rho0, p0, up):
    """Gas at rest (rho0, p0) pushed by a piston moving at speed up > 0.

    Mass and momentum across the shock moving at S give rho1 (S - up) = rho0 S and
    p1 - p0 = rho0 S up; the energy jump closes the system with
    S^2 - (gamma+1)/2 up S - a0^2 = 0.  Returns (S, rho1, p1).
    """
    a0 = sound_speed(gamma, rho0, p0)
    k = (gamma + 1.0) * up / 4.0
    S = k + math.sqrt(k * k + a0 * a0)
    rho1 = rho0 * S / (S - up)
    p1 = p0 + rho0 * S * up
    return S, rho1, p1


def normal_shock(gamma, M):
    """Density and pressure ratios across a normal shock with upstream Mach number M."""
    r = (gamma + 1.0) * M * M / ((gamma - 1.0) * M * M + 2.0)
    pr = 1.0 + 2.0 * gamma * (M * M - 1.0) / (gamma + 1.0)
    return r, pr


def stationary_shock_downstream(gamma, rho1, u1, p1):
    """Downstream state of a stationary normal shock with upstream state (rho1, u1, p1)."""
    M = u1 / sound_speed(gamma, rho1, p1)
    r, pr = normal_shock(gamma, M)
    return rho1 * r, u1 / r, p1 * pr


def piston_from_shock_mach(gamma, rho0, p0, Ms):
    """Piston (post-shock) speed that drives a shock of Mach number Ms into gas at rest."""
    a0 = sound_speed(gamma, rho0, p0)
    S = Ms * a0
    r, _ = normal_shock(gamma, Ms)
    return S * (1.0 - 1.0 / r)


# ------------------------------------------------------------------ exact Riemann solver
def _f_branch(p, rhoK, pK, aK, gamma):
    """Velocity jump across the wave on side K as a function of the star pressure p, and
    its derivative: shock branch (Rankine-Hugoniot) for p > pK, isentrope otherwise."""
    if p > pK:
        A = 2.0 / ((gamma + 1.0) * rhoK)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        q = math.sqrt(A / (p + B))
        f = (p - pK) * q
        df = q * (1.0 - (p - pK) / (2.0 * (B + p)))
    else:
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * aK / (gamma - 1.0) * ((p / pK) ** e - 1.0)
        df = 1.0 / (rhoK * aK) * (p / pK) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def riemann_star(WL, WR, gamma=1.4, tol=1e-14, maxit=100):
    """Star-region pressure and velocity for left/right primitive states (rho, u, p)."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    al, ar = sound_speed(gamma, rl, pl), sound_speed(gamma, rr, pr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum generated")
    # two-rarefaction guess: positive and usually close
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) / (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-12 * min(pl, pr))
    for _ in range(maxit):
        fl, dfl = _f_branch(p, rl, pl, al, gamma)
        fr, dfr = _f_branch(p, rr, pr, ar, gamma)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_branch(p, rl, pl, al, gamma)
    fr, _ = _f_branch(p, rr, pr, ar, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(WL, WR, xi, gamma=1.4):
    """Exact solution (rho, u, p) at similarity coordinates xi = x/t (array)."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    al, ar = sound_speed(gamma, rl, pl), sound_speed(gamma, rr, pr)
    ps, us = riemann_star(WL, WR, gamma)
    g = gamma
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros((3,) + xi.shape)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                SL = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= SL:
                    w = (rl, ul, pl)
                else:
                    r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    w = (r, us, ps)
            else:  # left rarefaction
                ast = al * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= ul - al:
                    w = (rl, ul, pl)
                elif s >= us - ast:
                    w = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * al) * (ul - s)
                    r = rl * c ** (2 / (g - 1))
                    u = 2 / (g + 1) * (al + (g - 1) / 2 * ul + s)
                    p = pl * c ** (2 * g / (g - 1))
                    w = (r, u, p)
        else:  # right of contact
            if ps > pr:  # right shock
                SR = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= SR:
                    w = (rr, ur, pr)
                else:
                    r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                    w = (r, us, ps)
            else:  # right rarefaction
                ast = ar * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= ur + ar:
                    w = (rr, ur, pr)
                elif s <= us + ast:
                    w = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * ar) * (ur - s)
                    r = rr * c ** (2 / (g - 1))
                    u = 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
                    p = pr * c ** (2 * g / (g - 1))
                    w = (r, u, p)
        out[(0,) + idx], out[(1,) + idx], out[(2,) + idx] = w
    return out
