"""On-lattice velocity sets and their weights (Formulas (3)-(5), (9), (10);
Tables 2 and 3).

Test infrastructure: see the package docstring.

A velocity set is a union of symmetry groups: each group is the orbit of a
representative integer vector under coordinate permutations and sign changes
(the paragraph introducing G_1, G_4, G_8 in 2D and G_1 ... G_48 in 3D).  All
velocities of a group share one weight.  The discrete velocities of the
dimensionless formulation are v_i = c e_i with integer e_i; on the lattice the
particle displacement per step is e_i itself.

Canonical order (an interface convention, since the paper fixes none): groups
in table order, and inside a group the vectors sorted ascending as integer
tuples (e_x, e_y[, e_z]).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from .counting import partitions_at_most

# Table 2: 2D 33-velocity model.  (group order, representative, printed weight)
TABLE2 = [
    (1, (0, 0), 0.161987),
    (4, (1, 0), 0.143204),
    (4, (1, 1), 0.0338840),
    (4, (2, 0), 0.00556112),
    (4, (2, 2), 8.44799e-5),
    (4, (3, 0), 0.00113254),
    (8, (2, 1), 0.0128169),
    (4, (4, 4), 3.45552e-6),
]
TABLE2_C = 0.819381

# Table 3: 3D 95-velocity model.
TABLE3 = [
    (1, (0, 0, 0), 0.206847),
    (6, (2, 0, 0), 0.00442257),
    (12, (2, 2, 0), 0.0333341),
    (8, (2, 2, 2), 0.0128902),
    (6, (3, 0, 0), 0.0287920),
    (12, (3, 3, 0), 0.00264319),
    (8, (3, 3, 3), 0.000927908),
    (24, (2, 2, 5), 0.00106078),
    (12, (4, 4, 0), 0.000804376),
    (6, (5, 0, 0), 0.00274697),
]
TABLE3_C = 0.421803

TABLES = {"D2Q33": (TABLE2, TABLE2_C), "D3Q95": (TABLE3, TABLE3_C)}

# Accuracy order of the published models: m = 4, so Formula (5) runs up to
# n_max = 2m = 8 (the statement after Formula (8)).
ORDER_M = 4

# Lower-order 3D sets that the paper says the same construction gives (the
# paragraph after Formula (10)): order m = 2, so Formula (5) up to n_max = 4,
# Omega(2, 3) = 4 equations for three group weights and c (Formula (10)).
# The paper prints no weights for them; the solve starts from least squares
# at c = 1.  (group order, representative)
LOWER_ORDER = {
    "D3Q19": [(1, (0, 0, 0)), (6, (1, 0, 0)), (12, (1, 1, 0))],
    "D3Q15": [(1, (0, 0, 0)), (6, (1, 0, 0)), (8, (1, 1, 1))],
}
LOWER_ORDER_M = 2


def model_order(name: str) -> int:
    """Order of accuracy m of a model; its equilibrium has order N = m (the
    paragraph after Formula (5) requires N >= m)."""
    return LOWER_ORDER_M if name in LOWER_ORDER else ORDER_M


def group_table(name: str):
    """[(group order, representative)] of a model, in table order."""
    if name in LOWER_ORDER:
        return list(LOWER_ORDER[name])
    return [(o, r) for (o, r, _w) in TABLES[name][0]]


def orbit(rep: Tuple[int, ...]) -> List[Tuple[int, ...]]:
    """All images of ``rep`` under coordinate permutations and sign flips,
    without repetition, sorted ascending."""
    D = len(rep)
    pts = set()
    for perm in itertools.permutations(range(D)):
        for signs in itertools.product((1, -1), repeat=D):
            pts.add(tuple(signs[a] * rep[perm[a]] for a in range(D)))
    return sorted(pts)


def double_factorial(n: int) -> int:
    """n!! with (-1)!! = 0!! = 1."""
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


def gaussian_moment(a: Tuple[int, ...]) -> float:
    """Right-hand side of Formula (5) normalised so that the weights sum to 1.

    Formula (4) gives prod_alpha Gamma((a_alpha + 1)/2) for the integral of
    exp(-v^2) v^a; dividing by the zeroth moment pi^(D/2) (Tables 2 and 3
    print weights that sum to one) leaves prod_alpha (a_alpha - 1)!! / 2^(a_alpha/2)
    for all-even multi-indices, and zero otherwise.
    """
    if any(x % 2 for x in a):
        return 0.0
    out = 1.0
    for x in a:
        out *= double_factorial(x - 1) / 2.0 ** (x // 2)
    return out


def equation_indices(D: int, m: int = ORDER_M) -> List[Tuple[int, ...]]:
    """Even multi-indices of Formula (5) up to n_max = 2m, one per partition
    (isotropy makes the ordering of the exponents irrelevant)."""
    out = []
    for q in range(m + 1):
        for p in partitions_at_most(q, D):
            out.append(tuple(2 * x for x in p))
    return out


@dataclass
class VelocitySet:
    name: str
    D: int
    e: np.ndarray            # (Q, D) int64, canonical order
    group: np.ndarray        # (Q,) group index into the table
    group_sizes: List[int]
    W: np.ndarray            # (G,) group weights
    c: float
    m: int = ORDER_M         # order of accuracy; the equilibrium has order N = m

    @property
    def Q(self) -> int:
        return int(self.e.shape[0])

    @property
    def w(self) -> np.ndarray:
        return self.W[self.group]

    @property
    def T0(self) -> float:
        """Lattice temperature of the reference state, T0 = 1/(2 c^2).

        From v = Theta^(-1/2) V with Theta = 2 k_B T0 / m_g and v_i = c e_i,
        V_i = e_i on the lattice gives Theta = 1/c^2, hence T0 = 1/(2c^2) in
        units where k_B/m_g = 1.
        """
        return 1.0 / (2.0 * self.c * self.c)


def build_orbits(name: str):
    table = group_table(name)
    D = len(table[0][1])
    e_list, g_list = [], []
    for g, (order, rep) in enumerate(table):
        orb = orbit(rep)
        if len(orb) != order:
            raise AssertionError(f"{name} group {g}: orbit of {rep} has {len(orb)} points, table says {order}")
        e_list.extend(orb)
        g_list.extend([g] * len(orb))
    return D, np.array(e_list, dtype=np.int64), np.array(g_list, dtype=np.int64)


def orbit_moment_matrix(name: str, m: int = None):
    """B[k, g] = sum over the orbit of group g of prod_alpha e_alpha^(a_k alpha),
    and the order |a_k| of each equation (Formula (5) up to n_max = 2m, by
    default with the model's own m)."""
    if m is None:
        m = model_order(name)
    D, e, grp = build_orbits(name)
    idx = equation_indices(D, m)
    G = int(grp.max()) + 1
    B = np.zeros((len(idx), G))
    order = np.zeros(len(idx), dtype=np.int64)
    for k, a in enumerate(idx):
        mono = np.prod(e.astype(np.float64) ** np.array(a, dtype=np.float64), axis=1)
        for g in range(G):
            B[k, g] = mono[grp == g].sum()
        order[k] = sum(a)
    rhs = np.array([gaussian_moment(a) for a in idx])
    return idx, B, order, rhs


def residual(name: str, W: np.ndarray, c: float) -> np.ndarray:
    """Left minus right side of Formula (5), with v_i = c e_i."""
    _, B, order, rhs = orbit_moment_matrix(name)
    return (B * (c ** order)[:, None]) @ W - rhs


def solve_weights(name: str, tol: float = 1e-15, maxit: int = 60):
    """Newton iteration on the square system of Formula (5) for (W_1..W_G, c).

    The unknowns are the G group weights and the speed c (Formula (10):
    Omega(m, D) = 1 + number of groups).  Started from the printed table
    values, so it converges to the root the paper reports.  The iteration
    runs in float64 and is then continued at 40 decimal digits (mpmath), so
    the returned float64 values are the rounded exact root: the Jacobian's
    condition number (about 3e6) would otherwise leave errors near 1e-11.
    """
    import mpmath

    _, B, order, rhs = orbit_moment_matrix(name)
    G = B.shape[1]
    if B.shape[0] != G + 1:
        raise AssertionError("system is not square")
    if name in TABLES:
        table, c0 = TABLES[name]
        x = np.array([w for (_o, _r, w) in table] + [c0], dtype=np.float64)
    else:
        # no printed values: least-squares weights at c = 1
        c0 = 1.0
        W0, *_ = np.linalg.lstsq(B * (c0 ** order)[:, None], rhs, rcond=None)
        x = np.concatenate([W0, [c0]])
    for _ in range(maxit):
        W, c = x[:G], x[G]
        cp = c ** order
        F = (B * cp[:, None]) @ W - rhs
        J = np.zeros((G + 1, G + 1))
        J[:, :G] = B * cp[:, None]
        dcp = np.where(order > 0, order * c ** np.maximum(order - 1, 0), 0.0)
        J[:, G] = (B * dcp[:, None]) @ W
        dx = np.linalg.solve(J, -F)
        x = x + dx
        if np.max(np.abs(dx) / np.maximum(np.abs(x), 1e-300)) < tol:
            break
    with mpmath.workdps(40):
        xm = [mpmath.mpf(float(v)) for v in x]
        Bm = [[mpmath.mpf(float(b)) for b in row] for row in B]
        rm = [mpmath.mpf(float(r)) for r in rhs]
        for _ in range(4):
            W, c = xm[:G], xm[G]
            F = mpmath.matrix(G + 1, 1)
            J = mpmath.matrix(G + 1, G + 1)
            for k in range(G + 1):
                o = int(order[k])
                acc = mpmath.fsum(W[g] * Bm[k][g] for g in range(G))
                F[k] = c ** o * acc - rm[k]
                for g in range(G):
                    J[k, g] = c ** o * Bm[k][g]
                J[k, G] = (o * c ** (o - 1) if o > 0 else 0) * acc
            dx = mpmath.lu_solve(J, -F)
            xm = [xm[k] + dx[k] for k in range(G + 1)]
        x = np.array([float(v) for v in xm])
    return x[:G].copy(), float(x[G])


_CACHE: Dict[str, VelocitySet] = {}


def velocity_set(name: str) -> VelocitySet:
    """Canonical velocity set with weights and c solved to float64 precision."""
    if name not in _CACHE:
        D, e, grp = build_orbits(name)
        W, c = solve_weights(name)
        _CACHE[name] = VelocitySet(name, D, e, grp, [t[0] for t in group_table(name)], W, c,
                                   model_order(name))
    return _CACHE[name]
