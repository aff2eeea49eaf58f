"""Pins of the oracle's model construction: Table 1, Formulas (8)-(10), Tables 2-3,
and the weight equations (3)-(5) checked by independent quadrature."""
import itertools

import mpmath
import numpy as np
import pytest

from conftest import read_golden
from oracle import counting, velocity_sets as vs

MODELS = ["D2Q33", "D3Q95"]


def test_table1_omega_matches_paper():
    rows = read_golden("table1_omega.txt")
    for row in rows:
        vals = [int(x) for x in row.split()]
        D, printed = vals[0], vals[1:]
        assert [counting.omega(m, D) for m in range(8)] == printed


def test_omega_equals_brute_force_even_multi_indices():
    # Brute force: distinct even multi-indices of order <= 2m up to permutation.
    for D in range(1, 5):
        for m in range(0, 8):
            seen = set()
            for a in itertools.product(range(0, 2 * m + 1, 2), repeat=D):
                if sum(a) <= 2 * m:
                    seen.add(tuple(sorted(a)))
            assert len(seen) == counting.omega(m, D)


def test_partition_counts_against_enumeration():
    for D in range(1, 5):
        counts = counting.restricted_partition_counts(12, D)
        for q in range(13):
            assert counts[q] == len(counting.partitions_at_most(q, D))


def _golden_table(name):
    rows = read_golden(name)
    groups, c = [], None
    for r in rows:
        f = r.split()
        if f[0] == "c":
            c = float(f[1])
            continue
        order = int(f[1])
        rep = tuple(int(x) for x in f[2:-1])
        groups.append((order, rep, float(f[-1])))
    return groups, c


GOLDEN = {"D2Q33": "table2_d2q33.txt", "D3Q95": "table3_d3q95.txt"}


@pytest.mark.parametrize("name", MODELS)
def test_velocity_count_and_orbits(name):
    groups, _ = _golden_table(GOLDEN[name])
    v = vs.velocity_set(name)
    # Formula (9): n(v_i) = sum_k k n_k
    assert v.Q == sum(o for (o, _r, _w) in groups) == int(name[3:])
    # every velocity distinct, orbit sizes as the group labels say
    assert len({tuple(x) for x in v.e.tolist()}) == v.Q
    for g, (order, rep, _w) in enumerate(groups):
        members = v.e[v.group == g]
        assert len(members) == order
        # members are exactly the signed permutations of the representative
        assert sorted(tuple(sorted(abs(x) for x in m)) for m in members.tolist()) == \
            [tuple(sorted(abs(x) for x in rep))] * order
    assert np.all(v.e.sum(0) == 0)
    # Formula (10): unknowns = groups + 1 = Omega(4, D)
    assert len(groups) + 1 == counting.omega(4, v.D)
    # largest displacement: 4 cells in 2D, 5 in 3D
    assert np.abs(v.e).max() == (4 if v.D == 2 else 5)


@pytest.mark.parametrize("name", MODELS)
def test_weights_match_printed_tables(name):
    groups, c_printed = _golden_table(GOLDEN[name])
    v = vs.velocity_set(name)
    for g, (_o, _r, w_printed) in enumerate(groups):
        # six significant digits as printed
        assert abs(v.W[g] - w_printed) <= 6e-6 * abs(w_printed), (g, v.W[g], w_printed)
    assert abs(v.c - c_printed) <= 1e-6 * c_printed
    assert np.all(v.W > 0) and v.c > 0


def _gauss_moment_1d(k):
    # int exp(-x^2) x^k dx / sqrt(pi) by Gauss-Hermite quadrature (exact for k < 2n)
    x, wq = np.polynomial.hermite.hermgauss(20)
    return float(np.sum(wq * x ** k) / np.sqrt(np.pi))


@pytest.mark.parametrize("name", MODELS)
def test_weights_integrate_every_monomial_to_degree_8(name):
    # Formula (3) for all multi-indices (odd, even, any order of exponents),
    # with v_i = c e_i and the Gaussian moments from Gauss-Hermite quadrature.
    v = vs.velocity_set(name)
    vel = v.c * v.e.astype(np.float64)
    worst = 0.0
    for n in range(0, 9):
        for a in itertools.product(range(n + 1), repeat=v.D):
            if sum(a) != n:
                continue
            lhs = float(np.sum(v.w * np.prod(vel ** np.array(a), axis=1)))
            rhs = float(np.prod([_gauss_moment_1d(k) for k in a]))
            worst = max(worst, abs(lhs - rhs) / max(1.0, abs(rhs)))
    assert worst < 1e-13, worst


@pytest.mark.parametrize("name", MODELS)
def test_weights_fail_at_degree_10(name):
    # Negative control: the model is built to degree 8 only, so some degree-10
    # moment is not reproduced.
    v = vs.velocity_set(name)
    vel = v.c * v.e.astype(np.float64)
    errs = []
    for a in itertools.product(range(11), repeat=v.D):
        if sum(a) != 10:
            continue
        lhs = float(np.sum(v.w * np.prod(vel ** np.array(a), axis=1)))
        rhs = float(np.prod([_gauss_moment_1d(k) for k in a]))
        errs.append(abs(lhs - rhs) / max(1.0, abs(rhs)))
    assert max(errs) > 1e-3


@pytest.mark.parametrize("name", MODELS)
def test_float64_newton_matches_high_precision_root(name):
    # Re-solve Formula (5) at 40 digits with mpmath from the printed values,
    # building the system directly from the velocity list.
    mpmath.mp.dps = 40
    v = vs.velocity_set(name)
    groups, c_printed = _golden_table(GOLDEN[name])
    G = len(groups)
    idx = []
    for n in range(0, 9, 2):
        for a in itertools.product(range(0, n + 1, 2), repeat=v.D):
            if sum(a) == n and list(a) == sorted(a, reverse=True):
                idx.append(a)
    assert len(idx) == G + 1

    def rhs(a):
        out = mpmath.mpf(1)
        for k in a:
            out *= mpmath.gamma(mpmath.mpf(k + 1) / 2) / mpmath.sqrt(mpmath.pi)
        return out

    ev = v.e.tolist()
    grp = v.group.tolist()

    def system(*x):
        W, c = x[:G], x[G]
        out = []
        for a in idx:
            s = mpmath.mpf(0)
            for e, g in zip(ev, grp):
                term = W[g]
                for comp, k in zip(e, a):
                    term *= (c * comp) ** k
                s += term
            out.append(s - rhs(a))
        return out

    x0 = [mpmath.mpf(w) for (_o, _r, w) in groups] + [mpmath.mpf(c_printed)]
    root = mpmath.findroot(system, x0, tol=mpmath.mpf(10) ** -35)
    W_hp = np.array([float(root[g]) for g in range(G)])
    c_hp = float(root[G])
    # the oracle returns the float64 rounding of the root
    assert abs(v.c - c_hp) / c_hp <= 2 ** -53
    assert np.max(np.abs(v.W - W_hp) / W_hp) <= 2 ** -53


@pytest.mark.parametrize("name", MODELS)
def test_reference_temperature_reading(name):
    # T0 = 1/(2c^2) equals the discrete second moment sum_i w_i e_ix^2
    v = vs.velocity_set(name)
    m2 = float(np.sum(v.w * v.e[:, 0].astype(float) ** 2))
    assert abs(m2 - v.T0) < 1e-14 * v.T0 * 10
    assert abs(v.T0 - 1.0 / (2 * v.c ** 2)) < 1e-15 * v.T0
