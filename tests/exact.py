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


def crout_lu_rows(m: Sequence[Sequence], cols: Sequence[int]):
    """Exact LU without pivoting of the column-permuted matrix A[:, cols]:
    A[:, cols] = L U, L lower triangular (its diagonal holds the pivots),
    U unit upper triangular.  Rows are taken top to bottom.  Returns
    (pivots, U) with Fractions, or None if a zero pivot appears.  A
    textbook elimination, independent of condensation and of any pivot
    rule: the caller supplies the column order to be checked."""
    n = len(m)
    a = [[Fraction(m[i][c]) for c in cols] for i in range(n)]
    piv, urows = [], []
    for s in range(n):
        p = a[s][s]
        if p == 0:
            return None
        piv.append(p)
        urow = [Fraction(0)] * n
        urow[s] = Fraction(1)
        for j in range(s + 1, n):
            urow[j] = a[s][j] / p
        urows.append(urow)
        for i in range(s + 1, n):
            f = a[i][s]
            if f == 0:
                continue
            for j in range(s + 1, n):
                a[i][j] -= f * urow[j]
    return piv, urows


def satisfies_maxabs_rule(m: Sequence[Sequence], cols: Sequence[int]) -> bool:
    """True iff `cols` is the pivot-column sequence of the largest-|a| rule
    with ties to the smallest original column, rows top to bottom: in the
    exact factorisation A[:, cols] = L U (crout_lu_rows) every |U[s][j]| <= 1
    (the pivot is a largest entry of its condensed row) and |U[s][j]| == 1
    only where cols[s] < cols[j] (a tie goes to the smaller original index).
    Those conditions fix the sequence uniquely, one step at a time."""
    n = len(m)
    if sorted(cols) != list(range(n)):
        return False
    f = crout_lu_rows(m, cols)
    if f is None:
        return False
    _, u = f
    for s in range(n):
        for j in range(s + 1, n):
            a = abs(u[s][j])
            if a > 1 or (a == 1 and cols[s] > cols[j]):
                return False
    return True
