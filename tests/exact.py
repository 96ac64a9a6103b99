"""Exact-arithmetic references used to pin the oracle (tests only).

These are textbook definitions, independent of condensation: the Laplace
(cofactor) expansion, Bareiss fraction-free elimination on Python integers,
the adjugate inverse, and permutation parity by counting inversions.
"""

from __future__ import annotations

import math
from fractions import Fraction
from typing import List, Sequence


def _minor(m: List[List[int]], i: int, j: int) -> List[List[int]]:
    return [row[:j] + row[j + 1:] for k, row in enumerate(m) if k != i]


def cofactor_det(m: Sequence[Sequence]) -> int:
    """Laplace expansion along the first row (exact for ints/Fractions)."""
    m = [list(r) for r in m]
    n = len(m)
    if n == 0:
        return 1
    if n == 1:
        return m[0][0]
    total = 0
    for j in range(n):
        if m[0][j] == 0:
            continue
        sgn = -1 if j % 2 else 1
        total += sgn * m[0][j] * cofactor_det(_minor(m, 0, j))
    return total


def bareiss_det(m: Sequence[Sequence[int]]) -> int:
    """Bareiss fraction-free elimination; every division is exact."""
    a = [[int(x) for x in r] for r in m]
    n = len(a)
    if n == 0:
        return 1
    sign = 1
    prev = 1
    for k in range(n - 1):
        if a[k][k] == 0:
            sw = next((i for i in range(k + 1, n) if a[i][k] != 0), None)
            if sw is None:
                return 0
            a[k], a[sw] = a[sw], a[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                num = a[i][j] * a[k][k] - a[i][k] * a[k][j]
                assert num % prev == 0
                a[i][j] = num // prev
        prev = a[k][k]
    return sign * a[n - 1][n - 1]


def adjugate_inverse(m: Sequence[Sequence[int]]) -> List[List[Fraction]]:
    """A^{-1} = adj(A) / det(A) with exact cofactors."""
    m = [list(r) for r in m]
    n = len(m)
    d = cofactor_det(m)
    if d == 0:
        raise ZeroDivisionError("singular")
    inv = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            c = cofactor_det(_minor(m, j, i)) * (-1 if (i + j) % 2 else 1)
            inv[i][j] = Fraction(c, d)
    return inv


def perm_parity_inversions(p: Sequence[int]) -> int:
    """+1 / -1 by counting inversions (O(n^2))."""
    inv = 0
    n = len(p)
    for i in range(n):
        for j in range(i + 1, n):
            if p[i] > p[j]:
                inv += 1
    return -1 if inv % 2 else 1


def log_abs_int(d: int) -> float:
    return math.log(abs(d))
