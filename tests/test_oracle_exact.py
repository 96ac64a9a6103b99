"""Pins of the oracle against exact arithmetic and the paper's own examples.

The oracle (oracle/mc_oracle.c) is checked here against things it does not
share code with: the Laplace expansion and Bareiss elimination on integer
matrices, the one-step identity of Eq. 1-3 in exact integers, and the worked
examples of Section 2.2 and Figure 3.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


# --- whole result vs exact determinants --------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_cofactor_expansion_integer(n):
    """sign exact, log|det| to ~1e-13 against the Laplace expansion."""
    checked = 0
    for seed in range(40 if n <= 6 else 6):
        a = synth.int_matrix(n, 1000 * n + seed)
        d = exact.cofactor_det(a.astype(int).tolist())
        if d == 0:
            continue
        r = O.slogdet(a)
        assert r.info == 0
        assert r.sign == (1 if d > 0 else -1), (n, seed, d)
        assert _rel(r.logabsdet, exact.log_abs_int(d)) < 1e-12
        checked += 1
    assert checked > 0


@pytest.mark.parametrize("n", [10, 16, 24, 33, 48, 64])
def test_bareiss_integer(n):
    for seed in range(3):
        a = synth.int_matrix(n, 7000 + 10 * n + seed)
        d = exact.bareiss_det(a.astype(int).tolist())
        assert d != 0
        r = O.slogdet(a)
        assert r.sign == (1 if d > 0 else -1)
        assert _rel(r.logabsdet, exact.log_abs_int(d)) < 1e-11


def test_bareiss_matches_cofactor():
    """The two exact references agree with each other (n <= 7)."""
    for n in range(1, 8):
        a = synth.int_matrix(n, 42 + n).astype(int).tolist()
        assert exact.bareiss_det(a) == exact.cofactor_det(a)


def test_exact_ties_and_negatives():
    """Matrices with many tied |entries| (entries in {-1, 0, 1, 2, -2})."""
    for seed in range(60):
        n = 2 + seed % 7
        a = synth.int_matrix(n, 9000 + seed, lo=-2, hi=2)
        d = exact.cofactor_det(a.astype(int).tolist())
        r = O.slogdet(a)
        if d == 0:
            # rounding may leave a tiny pivot instead of an exact zero
            assert r.sign == 0 or r.logabsdet < -20
            continue
        assert r.sign == (1 if d > 0 else -1)
        assert _rel(r.logabsdet, exact.log_abs_int(d)) < 1e-12


# --- one condensation step (Eq. 1, 2, 3) -------------------------------------

@pytest.mark.parametrize("n", [3, 4, 5, 6, 7])
def test_eq2_step_identity_exact(n):
    """det A * a_kl^(N-2) * (-1)^(k+l) == det B for every pivot (k, l).

    Integer A keeps B (products of small integers) exact, so both sides
    are exact integers.  The (-1)^(k+l) factor is absent from Eq. 1 as
    printed; the identity needs it."""
    a = synth.int_matrix(n, 300 + n)
    ai = a.astype(int).tolist()
    det_a = exact.cofactor_det(ai)
    for k in range(n):
        for l in range(n):
            akl = ai[k][l]
            if akl == 0:
                continue
            b = O.condense_step(a, k, l)
            bi = [[int(round(x)) for x in row] for row in b]
            assert np.array_equal(b, np.array(bi, dtype=np.float64))
            det_b = exact.cofactor_det(bi)
            assert det_b == (-1) ** (k + l) * det_a * akl ** (n - 2)


def test_eq1_as_printed_needs_sign_factor():
    """Without (-1)^(k+l) the printed Eq. 1 fails for odd k+l."""
    a = synth.int_matrix(4, 77)
    ai = a.astype(int).tolist()
    det_a = exact.cofactor_det(ai)
    assert det_a != 0
    k, l = 0, 1
    b = O.condense_step(a, k, l)
    det_b = exact.cofactor_det([[int(round(x)) for x in r] for r in b])
    assert det_b * 1 != det_a * ai[k][l] ** 2
    assert det_b == -det_a * ai[k][l] ** 2


@pytest.mark.parametrize("n", [3, 5, 7])
def test_eq3_factored_step(n):
    """det A = (-1)^(k+l) a_kl det B* with the pivot factored out of row k
    (Eq. 3, Section 2.3), checked in floating point against Laplace."""
    a = synth.int_matrix(n, 500 + n)
    ai = a.astype(int).tolist()
    det_a = exact.cofactor_det(ai)
    for k in range(n):
        for l in range(n):
            if ai[k][l] == 0:
                continue
            bstar = O.condense_step(a, k, l, factored=True)
            lhs = (-1) ** (k + l) * ai[k][l] * np.linalg.det(bstar)
            assert abs(lhs - det_a) <= 1e-9 * max(1, abs(det_a))


def test_eq3_equals_eq2_over_pivot():
    """B* = B / a_kl entrywise, to rounding (Eq. 3 vs Eq. 2)."""
    a = synth.uniform(6, 3)
    for k, l in [(0, 0), (2, 4), (5, 1)]:
        b = O.condense_step(a, k, l)
        bs = O.condense_step(a, k, l, factored=True)
        np.testing.assert_allclose(bs, b / a[k, l], rtol=1e-13, atol=1e-15)


# --- the paper's worked examples ---------------------------------------------

def test_fig3_large_pivot_bitwise():
    g = _load("fig3_large_pivot.json")
    a = np.array(g["A"], dtype=np.float64)
    bstar = O.condense_step(a, g["pivot_row"], g["pivot_col"], factored=True)
    assert np.array_equal(bstar, np.array(g["B_star"], dtype=np.float64))
    # the full loop starting from the same pivot row gives det A = e det B*
    r = O.slogdet(a, rows=O.ROWS_EXPLICIT, row_order=[1, 0, 2], pivots=True)
    assert r.piv_col[0] == g["pivot_col"]
    expect = math.log(g["logabsdet_terms"]["log_e"]) + math.log(
        g["logabsdet_terms"]["abs_det_B_star"])
    assert _rel(r.logabsdet, expect) < 1e-15
    assert r.sign == g["sign"]
    # and top-down order gives the same determinant
    r2 = O.slogdet(a)
    assert r2.sign == g["sign"] and _rel(r2.logabsdet, expect) < 1e-15


def test_sec22_pivot_rule_choice():
    g = _load("sec22_pivot_rule.json")
    row = np.array(g["row"])
    n = row.size
    a = np.eye(n)
    a[0] = row
    for rule, key in [(O.COL_MAXABS, "maxabs_choice"),
                      (O.COL_CLOSEST_TO_ONE, "closest_to_one_choice")]:
        r = O.slogdet(a, col_rule=rule, pivots=True)
        assert r.piv_col[0] == g[key]


def test_sec22_tiny_pivot_loses_accuracy():
    """The Section 2.2 argument, quantified: on a row of {1e-10, 2.01}
    entries the closest-to-1 rule divides by 1e-10 and loses digits that
    the largest-|a| rule keeps."""
    rng = np.random.default_rng(5)
    n = 6
    errs = {O.COL_MAXABS: 0.0, O.COL_CLOSEST_TO_ONE: 0.0}
    for trial in range(20):
        # rows of tiny and just-above-2 entries, with a little noise so the
        # matrix stays well conditioned; the exact reference is the Laplace
        # expansion over the rational values of the stored doubles
        a = rng.choice([1e-10, 2.01, -2.01, -1e-10], size=(n, n)) \
            + 1e-3 * rng.standard_normal((n, n))
        from fractions import Fraction
        d = exact.cofactor_det([[Fraction(float(x)) for x in r] for r in a])
        ref = math.log(abs(d))
        for rule in errs:
            r = O.slogdet(a, col_rule=rule)
            errs[rule] = max(errs[rule], _rel(r.logabsdet, ref))
    assert errs[O.COL_MAXABS] < 1e-13
    assert errs[O.COL_CLOSEST_TO_ONE] > 100 * errs[O.COL_MAXABS]


def test_tie_break_smallest_original_column():
    a = np.array([[3.0, -3.0, 1.0, 3.0],
                  [1.0, 2.0, 0.5, 0.25],
                  [0.0, 1.0, 4.0, 1.0],
                  [2.0, 0.0, 1.0, 5.0]])
    r = O.slogdet(a, pivots=True)
    assert r.piv_col[0] == 0
    d = exact.cofactor_det([[__import__("fractions").Fraction(x) for x in row]
                            for row in a])
    assert r.sign == (1 if d > 0 else -1)
    assert _rel(r.logabsdet, math.log(abs(d))) < 1e-14


# --- special cases ------------------------------------------------------------

def test_empty_and_one_by_one():
    r = O.slogdet(np.zeros((0, 0)))
    assert (r.sign, r.logabsdet, r.info) == (1.0, 0.0, 0)
    for v in [3.5, -0.25, 1e-300, -7e200]:
        r = O.slogdet(np.array([[v]]))
        assert r.sign == math.copysign(1, v)
        assert r.logabsdet == math.log(abs(v))
    r = O.slogdet(np.array([[0.0]]))
    assert (r.sign, r.logabsdet, r.info) == (0.0, -math.inf, 1)


def test_two_by_two_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(200):
        a = rng.integers(-50, 51, (2, 2)).astype(float)
        d = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
        r = O.slogdet(a)
        if d == 0:
            continue
        assert r.sign == np.sign(d)
        assert _rel(r.logabsdet, math.log(abs(d))) < 1e-14


def test_singular_structural():
    a = synth.uniform(7, 1)
    z = a.copy()
    z[3] = 0.0
    r = O.slogdet(z)
    assert r.sign == 0 and r.logabsdet == -math.inf and r.info == 4
    zc = a.copy()
    zc[:, 5] = 0.0
    r = O.slogdet(zc)
    assert r.sign == 0 and r.logabsdet == -math.inf and r.info == 7
    r = O.slogdet(np.zeros((4, 4)))
    assert r.info == 1


def test_nonfinite_inputs():
    a = synth.uniform(6, 2)
    for bad in [np.nan, np.inf, -np.inf]:
        for pos in [(0, 0), (3, 2), (5, 5)]:
            b = a.copy()
            b[pos] = bad
            r = O.slogdet(b)
            assert r.info == O.INFO_NONFINITE
            assert math.isnan(r.logabsdet) and r.sign == 0


def test_argument_errors():
    lib = O.lib()
    res = O._Result()
    import ctypes
    assert lib.mco_slogdet(None, 3, 3, 0, None, 0, 0, ctypes.byref(res), None,
                           None, None) < 0
    a = np.eye(3)
    p = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.mco_slogdet(p, -1, 3, 0, None, 0, 0, ctypes.byref(res), None,
                           None, None) < 0
    assert lib.mco_slogdet(p, 3, 2, 0, None, 0, 0, ctypes.byref(res), None,
                           None, None) < 0
    with pytest.raises(ValueError):
        O.slogdet(a, rows=O.ROWS_EXPLICIT, row_order=[0, 0, 1])
    with pytest.raises(ValueError):
        O.slogdet(a, rows=O.ROWS_FIG6, n_virt=2)


def test_strided_input():
    a = synth.uniform(40, 9)
    big = np.full((40, 57), np.nan)
    big[:, :40] = a
    lib = O.lib()
    import ctypes
    res = O._Result()
    big = np.ascontiguousarray(big)
    rc = lib.mco_slogdet(big.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         40, 57, 0, None, 0, 0, ctypes.byref(res), None, None,
                         None)
    assert rc == 0
    r = O.slogdet(a)
    assert res.logabsdet == r.logabsdet and res.sign == r.sign


def test_partial_steps():
    a = synth.uniform(30, 4)
    r = O.slogdet_steps(a, 10)
    assert r.info == O.INFO_PARTIAL
    full = O.slogdet(a, pivots=True)
    assert _rel(r.logabsdet, float(np.sum(np.log(np.abs(full.piv_val[:10]))))) \
        < 1e-14
    assert O.slogdet_steps(a, 0).logabsdet == full.logabsdet
