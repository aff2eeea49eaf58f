"""Exact solution of the Riemann problem of the Euler equations for an ideal gas.

Test infrastructure: see the package docstring.

The paper validates its 3D model on a shock tube and compares the density and
temperature plateaus with "the analytical solution of the Riemann problem".
This module is that analytical solution, the textbook exact solver (two
nonlinear waves, star-region pressure from the root of the pressure function,
then sampling at x/t).  The gas is the monatomic ideal gas of the BGK model,
gamma = (D + 2) / D, with pressure p = rho T in lattice units.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class StarState:
    p: float
    u: float
    rho_l: float
    rho_r: float


def _f_k(p, rho, pk, gamma):
    """Pressure function of one side and its derivative."""
    a = math.sqrt(gamma * pk / rho)
    if p > pk:    # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    return (2.0 * a / (gamma - 1.0)) * ((p / pk) ** e - 1.0), (1.0 / (rho * a)) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))


def star_state(left, right, gamma) -> StarState:
    """Star-region pressure, velocity and densities for states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    du = ur - ul
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= du:
        raise ValueError("vacuum is generated")
    # initial guess: two-rarefaction approximation
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * du) / (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-12)
    for _ in range(200):
        fl, dl = _f_k(p, rl, pl, gamma)
        fr, dr = _f_k(p, rr, pr, gamma)
        g = fl + fr + du
        pn = p - g / (dl + dr)
        if pn <= 0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_k(p, rl, pl, gamma)
    fr, _ = _f_k(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    gm = (gamma - 1.0) / (gamma + 1.0)
    if p > pl:
        rho_l = rl * (p / pl + gm) / (gm * p / pl + 1.0)
    else:
        rho_l = rl * (p / pl) ** (1.0 / gamma)
    if p > pr:
        rho_r = rr * (p / pr + gm) / (gm * p / pr + 1.0)
    else:
        rho_r = rr * (p / pr) ** (1.0 / gamma)
    return StarState(p, u, rho_l, rho_r)


def wave_speeds(left, right, gamma):
    """(left head, left tail, right tail, right head) speeds; for a shock the
    head and tail coincide with the shock speed."""
    rl, ul, pl = left
    rr, ur, pr = right
    st = star_state(left, right, gamma)
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    if st.p > pl:
        sl = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * st.p / pl + (gamma - 1) / (2 * gamma))
        lh = lt = sl
    else:
        lh = ul - al
        lt = st.u - al * (st.p / pl) ** ((gamma - 1) / (2 * gamma))
    if st.p > pr:
        sr = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * st.p / pr + (gamma - 1) / (2 * gamma))
        rh = rt = sr
    else:
        rh = ur + ar
        rt = st.u + ar * (st.p / pr) ** ((gamma - 1) / (2 * gamma))
    return lh, lt, rt, rh


def sample(left, right, gamma, xi):
    """(rho, u, p) of the self-similar solution at xi = (x - x0) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    st = star_state(left, right, gamma)
    lh, lt, rt, rh = wave_speeds(left, right, gamma)
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    g1 = gamma - 1.0
    g2 = gamma + 1.0
    for k, s in np.ndenumerate(xi):
        if s < st.u:  # left of the contact
            if s < lh:
                rho[k], u[k], p[k] = rl, ul, pl
            elif s < lt:   # inside the left fan (lh < lt only for a rarefaction)
                b = 2.0 / g2 + g1 / (g2 * al) * (ul - s)
                rho[k] = rl * b ** (2.0 / g1)
                u[k] = 2.0 / g2 * (al + 0.5 * g1 * ul + s)
                p[k] = pl * b ** (2.0 * gamma / g1)
            else:
                rho[k], u[k], p[k] = st.rho_l, st.u, st.p
        else:
            if s > rh:
                rho[k], u[k], p[k] = rr, ur, pr
            elif s > rt:
                b = 2.0 / g2 - g1 / (g2 * ar) * (ur - s)
                rho[k] = rr * b ** (2.0 / g1)
                u[k] = 2.0 / g2 * (-ar + 0.5 * g1 * ur + s)
                p[k] = pr * b ** (2.0 * gamma / g1)
            else:
                rho[k], u[k], p[k] = st.rho_r, st.u, st.p
    return rho, u, p


def monatomic_gamma(D: int) -> float:
    """gamma = (D + 2) / D of a gas with D translational degrees of freedom."""
    return (D + 2.0) / D
