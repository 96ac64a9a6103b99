"""Pins of the oracle's pivot sequence and of its compensated log sum.

The pivot rule of Section 2.2 (Figure 6 step 4.1): in each condensed pivot
row take the column of largest |a|; ties go to the smallest original column
index (the reading this project takes where the paper is silent).  It is
pinned by a characterisation that does not run the condensation: for a
column order sigma, the exact factorisation A[:, sigma] = L U (rows top to
bottom, no pivoting, Fractions) must have |U[s][j]| <= 1 for j > s, with
equality only where sigma[s] < sigma[j].  Exactly one sigma satisfies that,
step by step.

Inputs where the arithmetic is exact in FP64 make the comparison exact:
totally unimodular matrices (every condensed entry stays in {-1, 0, 1}, so
about four steps in five are ties), and small random matrices whose
pivots are not near-tied (checked with the oracle's own gap output).

The log-sum pin: Figure 6 step 4.4 sums log|pivot|; a running sum that
grows large and then cancels loses ~1e-11 in a plain FP64 sum, while the
compensated sum must stay within a couple of ulps of the exactly rounded
sum of the same terms (math.fsum).
"""

import math

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import exact


@pytest.mark.parametrize("n", [2, 5, 12, 30, 48])
def test_unimodular_pivots_satisfy_the_rule_exactly(n):
    for seed in range(6):
        a = synth.unimodular_ties(n, 100 * n + seed)
        r, gap = O.slogdet_gaps(a)
        assert r.info == 0 and r.logabsdet == 0.0 and abs(r.sign) == 1.0
        cols = [int(c) for c in r.piv_col]
        assert exact.satisfies_maxabs_rule(a.astype(int).tolist(), cols), (n, seed)
        # the determinant of a unimodular matrix is +-1: the sign from the
        # exact pivots and the column order
        piv, _ = exact.crout_lu_rows(a.astype(int).tolist(), cols)
        d = exact.perm_parity_inversions(cols) * math.prod(int(p) for p in piv)
        assert d == exact.bareiss_det(a.astype(int).tolist()) == r.sign


def test_unimodular_has_ties_the_rule_must_break():
    """The family is worth testing with: most steps are exact ties."""
    a = synth.unimodular_ties(200, 5)
    _, gap = O.slogdet_gaps(a)
    assert set(np.unique(gap)) <= {0.0, 1.0}
    assert (gap == 0.0).mean() > 0.5


@pytest.mark.parametrize("n", [3, 8, 14])
def test_random_pivots_satisfy_the_rule_exactly(n):
    """Random real matrices, judged on the exact rationals of their FP64
    entries: where no step of the oracle's run is near-tied (gap > 1e-8)
    rounding cannot have changed a choice, and the FP64 sequence must be
    the exact one."""
    checked = 0
    for seed in range(8):
        a = synth.normal(n, 4000 + 10 * n + seed)
        r, gap = O.slogdet_gaps(a)
        if gap.min() <= 1e-8:
            continue
        cols = [int(c) for c in r.piv_col]
        assert exact.satisfies_maxabs_rule(a.tolist(), cols), (n, seed)
        checked += 1
    assert checked >= 4


def test_rule_characterisation_rejects_other_orders():
    """The characterisation is sharp: the same matrix with the sequence a
    different rule takes (Beliakov's first non-zero, Haque's closest to one,
    the largest original index among ties) fails it."""
    a = synth.unimodular_ties(24, 3)
    m = a.astype(int).tolist()
    good = [int(c) for c in O.slogdet(a, pivots=True).piv_col]
    assert exact.satisfies_maxabs_rule(m, good)
    b = synth.normal(10, 77)
    for rule in (O.COL_FIRST_NONZERO, O.COL_CLOSEST_TO_ONE):
        other = [int(c) for c in O.slogdet(b, col_rule=rule, pivots=True).piv_col]
        assert not exact.satisfies_maxabs_rule(b.tolist(), other)
    # reverse the tie-break by hand: the first step's tied column with the
    # largest index instead of the smallest
    row0 = np.abs(a[0])
    tied = np.flatnonzero(row0 == row0.max())
    assert len(tied) > 1
    assert good[0] == tied.min()
    assert not exact.satisfies_maxabs_rule(m, [int(tied.max())] + [
        c for c in range(24) if c != tied.max()])


def test_gap_output_matches_the_exact_rows():
    """gap[s] is 1 where the exact U row s has no other entry of magnitude
    1 beyond the pivot, and 0 where it has one (a tie)."""
    a = synth.unimodular_ties(40, 9)
    r, gap = O.slogdet_gaps(a)
    cols = [int(c) for c in r.piv_col]
    _, u = exact.crout_lu_rows(a.astype(int).tolist(), cols)
    for s in range(40):
        tie = any(abs(u[s][j]) == 1 for j in range(s + 1, 40))
        assert gap[s] == (0.0 if tie else 1.0), s
    b = synth.uniform(30, 8)
    rb, gb = O.slogdet_gaps(b)
    pv = O.slogdet(b, pivots=True)
    assert np.array_equal(rb.piv_col, pv.piv_col)
    assert (gb > 0).all() and (gb <= 1).all() and gb[-1] == 1.0


def test_threads_do_not_change_results():
    a = synth.normal(400, 31)
    prev = O.set_threads(1)
    try:
        r1 = O.slogdet(a, pivots=True)
        O.set_threads(4)
        r4 = O.slogdet(a, pivots=True)
    finally:
        O.set_threads(prev)
    assert r1.logabsdet == r4.logabsdet and r1.sign == r4.sign
    assert np.array_equal(r1.piv_col, r4.piv_col)
    assert np.array_equal(r1.piv_val, r4.piv_val)


def cancelling_diagonal(k: int = 300, seed: int = 2203):
    """diag(1e300 u_1 .. 1e300 u_k, 1e-300 / u_k .. 1e-300 / u_1, e): the
    log sum climbs to ~2e5 and falls back to ~1 in step order."""
    u = np.random.default_rng(seed).uniform(1.0, 2.0, k)
    d = np.concatenate([1e300 * u, 1e-300 / u[::-1], [math.e]])
    return np.diag(d), d


def test_log_sum_is_compensated():
    a, d = cancelling_diagonal()
    terms = [math.log(abs(x)) for x in d]  # the same libm log as the oracle
    exact_sum = math.fsum(terms)
    plain = 0.0
    for t in terms:
        plain += t
    assert abs(plain - exact_sum) > 1e-12  # the check has teeth
    r = O.slogdet(a)
    assert r.sign == 1.0
    assert abs(r.logabsdet - exact_sum) <= 4e-16 * max(1.0, abs(exact_sum))
