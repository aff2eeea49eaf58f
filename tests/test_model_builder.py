"""The library's general model constructor (Formulas (5) and (8)-(10)):
equation counts against Table 1, the paper's two models rebuilt from their
table representatives, and lower-order on-lattice sets whose weights and
reference temperature have closed forms.  Host-only (no device call)."""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import velocity_sets as ovs
from paper_1303_4624_amd import _lib as L


def test_equation_counts_match_table1():
    rows = read_golden("table1_omega.txt")
    assert len(rows) == 4
    for line in rows:
        row = line.split()
        D, counts = int(row[0]), [int(x) for x in row[1:]]
        assert [L.lbm_equation_count(m, D) for m in range(8)] == counts


@pytest.mark.parametrize("name,D", [("D2Q33", 2), ("D3Q95", 3)])
@pytest.mark.parametrize("with_guess", [True, False])
def test_tables_2_and_3_rebuilt_bit_for_bit(name, D, with_guess):
    table, c_printed = ovs.TABLES[name]
    reps = [r for (_o, r, _w) in table]
    wg = [w for (_o, _r, w) in table] if with_guess else None
    e, grp, w, c, res = L.lbm_model_build(D, 4, reps, c_printed, wg)
    e0, w0, c0 = L.lbm_velocity_set(D, len(e))
    assert np.array_equal(e, e0) and np.array_equal(w, w0) and c == c0
    assert [int(np.sum(grp == g)) for g in range(len(table))] == [o for (o, _r, _w) in table]
    assert res <= 1e-14


# Second-order sets (m = 2, Omega = 3 in 1D and 4 in 2D/3D): the solution is
# the familiar one with c_s^2 = T0 = 1/3, i.e. c = sqrt(3/2).
@pytest.mark.parametrize("D,Q,reps,weights", [
    (1, 3, [[0], [1]], [2 / 3, 1 / 6]),
    (2, 9, [[0, 0], [1, 0], [1, 1]], [4 / 9, 1 / 9, 1 / 36]),
    (3, 15, [[0, 0, 0], [1, 0, 0], [1, 1, 1]], [2 / 9, 1 / 9, 1 / 72]),
    (3, 19, [[0, 0, 0], [1, 0, 0], [1, 1, 0]], [1 / 3, 1 / 18, 1 / 36]),
])
def test_lower_order_sets_have_their_closed_forms(D, Q, reps, weights):
    e, grp, w, c, res = L.lbm_model_build(D, 2, reps, 1.0)
    assert len(e) == Q
    for g, wg in enumerate(weights):
        assert np.allclose(w[grp == g], wg, rtol=4e-16, atol=0)
    assert abs(c - math.sqrt(1.5)) <= 4e-16 * c
    assert abs(w.sum() - 1) <= 1e-15 and res <= 1e-15


def test_one_dimensional_five_velocity_set_has_two_roots():
    # {0, +-1, +-3} at m = 3: T0 = 1 +- sqrt(2/5); with the weights fixed by
    # sum w e^2 = T0 and sum w e^4 = 3 T0^2.
    found = set()
    for c_guess in (0.5, 1.0):
        e, grp, w, c, res = L.lbm_model_build(1, 3, [[0], [1], [3]], c_guess)
        T0 = 1 / (2 * c * c)
        root = min((1 - math.sqrt(0.4), 1 + math.sqrt(0.4)), key=lambda r: abs(r - T0))
        assert abs(T0 - root) <= 1e-14
        w3 = (3 * T0 * T0 - T0) / 144
        w1 = (T0 - 18 * w3) / 2
        assert abs(w[grp == 2][0] - w3) <= 1e-14 and abs(w[grp == 1][0] - w1) <= 1e-14
        found.add(round(root, 6))
    assert len(found) == 2


def test_constructor_rejections():
    cases = [
        # D3Q27's groups give 5 unknowns: 4 equations at m = 2, 7 at m = 3
        ((3, 2, [[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]], 1.0), L.LBM_E_INVALID),
        ((3, 3, [[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]], 1.0), L.LBM_E_INVALID),
        # two representatives of one group
        ((2, 2, [[0, 0], [1, 0], [0, -1]], 1.0), L.LBM_E_INVALID),
        # no velocity off the axes: the mixed moment e_x^2 e_y^2 cannot match
        ((2, 2, [[0, 0], [1, 0], [2, 0]], 1.0), L.LBM_E_INVALID),
        # solvable, but with a negative weight
        ((2, 3, [[0, 0], [1, 0], [2, 0], [3, 0], [2, 1]], 1.0), L.LBM_E_INVALID),
        ((4, 2, [[0, 0, 0, 0], [1, 0, 0, 0], [1, 1, 0, 0]], 1.0), L.LBM_E_UNSUPPORTED),
        ((2, 2, [[0, 0], [1, 0], [1, 1]], -1.0), L.LBM_E_INVALID),
    ]
    for args, want in cases:
        with pytest.raises(L.LBMError) as ex:
            L.lbm_model_build(*args)
        assert ex.value.status == want, args
    with pytest.raises(L.LBMError) as ex:
        L.lbm_equation_count(-1, 2)
    assert ex.value.status == L.LBM_E_INVALID
