"""Counting of moment equations by integer partitions (Formulas (6)-(8), Table 1).

Test infrastructure: see the package docstring.
"""
from __future__ import annotations

from typing import List, Tuple


def restricted_partition_counts(qmax: int, D: int) -> List[int]:
    """pi(q, D) for q = 0..qmax via the generating function of Formula (7).

    The product over k = 1..D of 1/(1 - x^k) is expanded as a product of
    truncated geometric series; the coefficient of x^q is the number of
    partitions of q into at most D parts (equivalently, with parts <= D, by
    conjugating the Ferrers graph).
    """
    series = [1] + [0] * qmax          # the constant series 1
    for k in range(1, D + 1):
        geom = [1 if q % k == 0 else 0 for q in range(qmax + 1)]   # 1/(1-x^k)
        prod = [0] * (qmax + 1)
        for i, a in enumerate(series):
            if a == 0:
                continue
            for j in range(0, qmax + 1 - i):
                if geom[j]:
                    prod[i + j] += a * geom[j]
        series = prod
    return series


def omega(m: int, D: int) -> int:
    """Omega(m, D) = sum_{q=0}^{m} pi(q, D): number of equations of Formula (5)
    up to n_max = 2m (Formula (8))."""
    return sum(restricted_partition_counts(m, D))


def partitions_at_most(q: int, D: int) -> List[Tuple[int, ...]]:
    """All partitions of q into at most D parts, as non-increasing D-tuples
    padded with zeros.  Doubling every part gives the even multi-indices
    (a_1, ..., a_D) of order 2q that index the equations of Formula (5)."""
    out: List[Tuple[int, ...]] = []

    def rec(rest: int, maxpart: int, acc: List[int]) -> None:
        if len(acc) == D:
            if rest == 0:
                out.append(tuple(acc))
            return
        for p in range(min(rest, maxpart), -1, -1):
            rec(rest - p, p, acc + [p])

    rec(q, q, [])
    return out
