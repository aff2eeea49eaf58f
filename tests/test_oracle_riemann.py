"""Pins of the exact Riemann solution inside the rarefaction fans.

The shock-tube experiment compares the simulated density and temperature
profiles with the analytical solution of the Riemann problem.  The oracle's
sampler `riemann.sample` writes the fan as closed forms in xi = x/t; these
tests check it against relations it does not use itself:

* inside a left fan the flow is isentropic (p / rho^gamma of the left state),
  carries the Riemann invariant u + 2a/(gamma - 1) of the left state, and
  xi is the characteristic speed u - a through the origin; a right fan
  mirrors this with u - 2a/(gamma - 1) and xi = u + a;
* the solution is continuous at a fan's head (the outer state) and tail (the
  star state), and the head and tail speeds are the characteristic speeds
  u - a (u + a) of the two states the fan joins, with the star sound speed
  taken from the star density;
* outside the fans the outer and star states are returned, and a shock obeys
  the Rankine-Hugoniot conditions on either side.

A wrong exponent, sign or velocity term in the fan formulas moves at least
one of these far above the bars.  Cases: the paper's tube (left fan, right
shock), its mirror (left shock, right fan), two fans, and two shocks.
"""
import math

import numpy as np
import pytest

from oracle import riemann as rm

G53 = 5.0 / 3.0
CASES = {
    # (left (rho, u, p), right (rho, u, p), gamma)
    "tube_fan_shock": ((4.0, 0.0, 4.0), (1.0, 0.0, 1.0), G53),
    "mirror_shock_fan": ((1.0, 0.0, 1.0), (4.0, 0.0, 4.0), G53),
    "two_fans": ((1.0, -1.0, 0.6), (0.8, 1.2, 0.5), G53),
    "two_shocks": ((1.0, 1.5, 1.0), (0.7, -1.0, 0.8), 1.4),
    "two_fans_gamma2": ((1.0, -0.5, 0.7), (1.0, 0.5, 0.7), 2.0),
}


def _sound(rho, p, g):
    return math.sqrt(g * p / rho)


def _kinds(L, R, g):
    st = rm.star_state(L, R, g)
    return ("fan" if st.p <= L[2] else "shock"), ("fan" if st.p <= R[2] else "shock"), st


@pytest.mark.parametrize("name", sorted(CASES))
def test_fan_isentrope_riemann_invariant_and_characteristic(name):
    L, R, g = CASES[name]
    kl, kr, st = _kinds(L, R, g)
    lh, lt, rt, rh = rm.wave_speeds(L, R, g)
    checked = 0
    for side, kind, (a, b) in (("L", kl, (lh, lt)), ("R", kr, (rt, rh))):
        if kind != "fan":
            continue
        xi = np.linspace(a, b, 41)[1:-1]
        rho, u, p = rm.sample(L, R, g, xi)
        c = np.sqrt(g * p / rho)
        outer = L if side == "L" else R
        ao = _sound(outer[0], outer[2], g)
        s0 = outer[2] / outer[0] ** g
        np.testing.assert_allclose(p / rho ** g, s0, rtol=1e-12)
        if side == "L":
            np.testing.assert_allclose(u + 2 * c / (g - 1), outer[1] + 2 * ao / (g - 1),
                                       rtol=0, atol=1e-12)
            np.testing.assert_allclose(u - c, xi, rtol=0, atol=1e-12)
        else:
            np.testing.assert_allclose(u - 2 * c / (g - 1), outer[1] - 2 * ao / (g - 1),
                                       rtol=0, atol=1e-12)
            np.testing.assert_allclose(u + c, xi, rtol=0, atol=1e-12)
        checked += 1
    assert checked == {"fan": 1, "shock": 0}[kl] + {"fan": 1, "shock": 0}[kr]


@pytest.mark.parametrize("name", sorted(CASES))
def test_head_tail_speeds_and_continuity(name):
    L, R, g = CASES[name]
    kl, kr, st = _kinds(L, R, g)
    lh, lt, rt, rh = rm.wave_speeds(L, R, g)
    aL, aR = _sound(L[0], L[2], g), _sound(R[0], R[2], g)
    a_sl = _sound(st.rho_l, st.p, g)     # star sound speeds from the star densities
    a_sr = _sound(st.rho_r, st.p, g)
    eps = 1e-7
    star_l = (st.rho_l, st.u, st.p)
    star_r = (st.rho_r, st.u, st.p)
    if kl == "fan":
        assert abs(lh - (L[1] - aL)) < 1e-13
        assert abs(lt - (st.u - a_sl)) < 1e-12
        assert lh < lt < st.u
        for x, want in ((lh - eps, L), (lh + eps, L), (lt - eps, star_l), (lt + eps, star_l)):
            got = [float(v[0]) for v in rm.sample(L, R, g, [x])]
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-6)
    else:
        assert lh == lt and lh < st.u
    if kr == "fan":
        assert abs(rh - (R[1] + aR)) < 1e-13
        assert abs(rt - (st.u + a_sr)) < 1e-12
        assert st.u < rt < rh
        for x, want in ((rh + eps, R), (rh - eps, R), (rt + eps, star_r), (rt - eps, star_r)):
            got = [float(v[0]) for v in rm.sample(L, R, g, [x])]
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-6)
    else:
        assert rh == rt and rh > st.u


@pytest.mark.parametrize("name", sorted(CASES))
def test_outer_and_star_states_and_shock_jumps(name):
    L, R, g = CASES[name]
    kl, kr, st = _kinds(L, R, g)
    lh, lt, rt, rh = rm.wave_speeds(L, R, g)
    xs = [lh - 1.0, 0.5 * (lt + st.u), 0.5 * (st.u + rt), rh + 1.0]
    rho, u, p = rm.sample(L, R, g, xs)
    want = [L, (st.rho_l, st.u, st.p), (st.rho_r, st.u, st.p), R]
    for k, w in enumerate(want):
        assert (rho[k], u[k], p[k]) == pytest.approx(w, rel=1e-14, abs=1e-14)
    # a shock: mass, momentum and energy fluxes continuous in its frame
    for kind, s, outer, rho_s in ((kl, lh, L, st.rho_l), (kr, rh, R, st.rho_r)):
        if kind != "shock":
            continue
        ro, uo, po = outer
        m_o, m_s = ro * (uo - s), rho_s * (st.u - s)
        assert abs(m_o - m_s) <= 1e-12 * abs(m_o)
        assert abs((m_o * (uo - s) + po) - (m_s * (st.u - s) + st.p)) <= 1e-12 * (po + st.p)
        h_o = g / (g - 1) * po / ro + 0.5 * (uo - s) ** 2
        h_s = g / (g - 1) * st.p / rho_s + 0.5 * (st.u - s) ** 2
        assert abs(h_o - h_s) <= 1e-12 * h_o


def test_fan_profile_is_monotone_and_self_similar():
    # Density falls and velocity rises monotonically through a left fan;
    # sampling at (x, t) and (2x, 2t) gives the same state.
    L, R, g = CASES["tube_fan_shock"]
    lh, lt, _, _ = rm.wave_speeds(L, R, g)
    xi = np.linspace(lh, lt, 50)
    rho, u, p = rm.sample(L, R, g, xi)
    assert np.all(np.diff(rho) < 0) and np.all(np.diff(u) > 0) and np.all(np.diff(p) < 0)
    x, t = np.linspace(-300, 300, 41), 120.0
    a = rm.sample(L, R, g, x / t)
    b = rm.sample(L, R, g, (2 * x) / (2 * t))
    for va, vb in zip(a, b):
        np.testing.assert_array_equal(va, vb)
