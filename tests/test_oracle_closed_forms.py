"""Pins of the oracle against closed-form determinants and invariants.

Closed forms: diagonal, triangular, Q diag(d) with Q a product of
Householder reflectors (det Q = (-1)^r), c I + u v^T, permutation matrices.
Invariants: det(AB) = det A det B, transpose, scaling, row/column swaps,
and independence from the order in which pivot rows are taken (Eq. 2 holds
for any k, Section 1 and Section 2.1), including the Figure 6 loop order.
Library cross-checks (numpy/scipy LAPACK) stand in as a special case: with
rows taken top-down the condensation is LU with partial pivoting of A^T.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import oracle as O
from tests import exact


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


@pytest.mark.parametrize("n", [1, 5, 64, 200])
def test_diagonal(n):
    rng = np.random.default_rng(n)
    d = rng.uniform(0.1, 10, n) * rng.choice([-1, 1], n)
    r = O.slogdet(np.diag(d))
    assert r.sign == np.prod(np.sign(d))
    assert _rel(r.logabsdet, float(np.sum(np.log(np.abs(d))))) < 1e-14


@pytest.mark.parametrize("n", [3, 12, 40])
@pytest.mark.parametrize("upper", [True, False])
def test_triangular(n, upper):
    """Off-diagonal entries larger than the diagonal force the max-|a| rule
    to pivot off the diagonal, yet det = prod(diag).  (Such matrices grow
    exponentially ill-conditioned with n, so the sizes stay small.)"""
    rng = np.random.default_rng(100 + n)
    t = rng.uniform(-3, 3, (n, n))
    d = rng.uniform(0.5, 2, n) * rng.choice([-1, 1], n)
    t = np.triu(t, 1) if upper else np.tril(t, -1)
    a = t + np.diag(d)
    r = O.slogdet(a)
    assert r.sign == np.prod(np.sign(d))
    assert _rel(r.logabsdet, float(np.sum(np.log(np.abs(d))))) < 1e-10


@pytest.mark.parametrize("n,refl", [(4, 1), (9, 2), (60, 3), (128, 7),
                                    (257, 10)])
def test_householder_q_diag(n, refl):
    a, d, r_ = synth.householder_qd(n, 31 * n + refl, refl)
    r = O.slogdet(a)
    assert r.sign == (-1) ** r_ * np.prod(np.sign(d))
    assert _rel(r.logabsdet, float(np.sum(np.log(np.abs(d))))) < 1e-12


@pytest.mark.parametrize("n", [2, 7, 50, 180])
def test_identity_plus_rank_one(n):
    """det(c I + u v^T) = c^(n-1) (c + v^T u)."""
    rng = np.random.default_rng(500 + n)
    for c in [1.5, -0.75]:
        u = rng.standard_normal(n)
        v = rng.standard_normal(n)
        a = c * np.eye(n) + np.outer(u, v)
        lam = c + float(v @ u)
        ref = (n - 1) * math.log(abs(c)) + math.log(abs(lam))
        sgn = (np.sign(c) ** (n - 1)) * np.sign(lam)
        r = O.slogdet(a)
        assert r.sign == sgn
        assert _rel(r.logabsdet, ref) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 8, 33, 100])
def test_permutation_matrices(n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        p = rng.permutation(n)
        a = np.zeros((n, n))
        a[np.arange(n), p] = 1.0
        r = O.slogdet(a)
        assert r.logabsdet == 0.0
        assert r.sign == exact.perm_parity_inversions(list(p))


# --- invariants ----------------------------------------------------------------

@pytest.mark.parametrize("n", [5, 37, 120])
def test_product_rule(n):
    a = synth.uniform(n, 10 + n)
    b = synth.normal(n, 20 + n)
    ra, rb, rab = O.slogdet(a), O.slogdet(b), O.slogdet(a @ b)
    assert rab.sign == ra.sign * rb.sign
    # a @ b is rounded: allow ~ cond * n * eps
    assert _rel(rab.logabsdet, ra.logabsdet + rb.logabsdet) < 1e-9


@pytest.mark.parametrize("n", [6, 45, 101])
def test_transpose_scaling_swaps(n):
    a = synth.normal(n, 3 * n)
    r = O.slogdet(a)
    rt = O.slogdet(a.T)
    assert rt.sign == r.sign and _rel(rt.logabsdet, r.logabsdet) < 1e-11
    for c in [2.0, -0.5]:  # powers of two: scaling is exact
        rc = O.slogdet(c * a)
        assert rc.sign == r.sign * (np.sign(c) ** n)
        assert _rel(rc.logabsdet, r.logabsdet + n * math.log(abs(c))) < 1e-12
    rs = O.slogdet(a[[1, 0] + list(range(2, n))])
    assert rs.sign == -r.sign and _rel(rs.logabsdet, r.logabsdet) < 1e-11
    cs = O.slogdet(a[:, [n - 1] + list(range(1, n - 1)) + [0]])
    assert cs.sign == -r.sign and _rel(cs.logabsdet, r.logabsdet) < 1e-11


@pytest.mark.parametrize("n", [8, 24, 64])
def test_pivot_row_independence(n):
    """Same determinant for top-down, bottom-up, random and Figure 6 row
    orders (Eq. 2 holds for any k)."""
    a = synth.uniform(n, 77 + n)
    ref = O.slogdet(a)
    rng = np.random.default_rng(n)
    runs = [O.slogdet(a, rows=O.ROWS_BOTTOM_UP),
            O.slogdet(a, rows=O.ROWS_EXPLICIT, row_order=rng.permutation(n)),
            O.slogdet(a, rows=O.ROWS_EXPLICIT, row_order=rng.permutation(n))]
    for nv in [2, 4, 8]:
        runs.append(O.slogdet(a, rows=O.ROWS_FIG6, n_virt=nv))
    for r in runs:
        assert r.info == 0
        assert r.sign == ref.sign
        assert _rel(r.logabsdet, ref.logabsdet) < 1e-12


def test_fig6_order_visits_block_rows():
    a = synth.uniform(8, 1)
    r = O.slogdet(a, rows=O.ROWS_FIG6, n_virt=4, pivots=True)
    assert list(r.piv_row) == [0, 2, 4, 6, 1, 3, 5, 7]


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_all_row_orders_brute_force(n):
    """Every one of the n! pivot-row orders yields the exact determinant."""
    a = synth.int_matrix(n, 60 + n)
    d = exact.cofactor_det(a.astype(int).tolist())
    assert d != 0
    for order in itertools.permutations(range(n)):
        r = O.slogdet(a, rows=O.ROWS_EXPLICIT, row_order=order)
        assert r.sign == (1 if d > 0 else -1)
        assert _rel(r.logabsdet, math.log(abs(d))) < 1e-13


def test_other_column_rules_same_determinant():
    """Beliakov's and Haque's pivot-column rules (Section 1) change the
    pivots, not the determinant, on well-conditioned integer input."""
    for n in [3, 5, 7]:
        a = synth.int_matrix(n, 880 + n)
        d = exact.cofactor_det(a.astype(int).tolist())
        for rule in [O.COL_FIRST_NONZERO, O.COL_CLOSEST_TO_ONE]:
            r = O.slogdet(a, col_rule=rule)
            assert r.sign == (1 if d > 0 else -1)
            assert _rel(r.logabsdet, math.log(abs(d))) < 1e-10


# --- library cross-checks (special case: LU with partial pivoting of A^T) ----

@pytest.mark.parametrize("n", [5, 50, 300])
def test_pivot_sequence_equals_lapack_on_transpose(n):
    a = synth.uniform(n, 4000 + n)
    r = O.slogdet(a, pivots=True)
    lu, ipiv = scipy.linalg.lu_factor(a.T)
    perm = list(range(n))
    chosen = []
    for s, p in enumerate(ipiv):
        perm[s], perm[p] = perm[p], perm[s]
        chosen.append(perm[s])
    assert list(r.piv_col) == chosen
    # the pivots are LAPACK's diagonal of U
    np.testing.assert_allclose(r.piv_val, np.diag(lu), rtol=1e-10)


@pytest.mark.parametrize("n", [1, 17, 256, 400])
def test_numpy_slogdet(n):
    a = synth.normal(n, 9 + n)
    r = O.slogdet(a)
    s, l = np.linalg.slogdet(a)
    assert r.sign == s
    assert _rel(r.logabsdet, l) < 1e-12


def test_wishart_input_is_spd():
    a = synth.wishart(64, 3)
    r = O.slogdet(a)
    s, l = np.linalg.slogdet(a)
    assert r.sign == 1.0 == s
    assert _rel(r.logabsdet, l) < 1e-12


# --- the explicit inverse (used to check gradients) ----------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_inverse_adjugate_exact(n):
    from fractions import Fraction
    a = synth.int_matrix(n, 123 + n)
    ai = a.astype(int).tolist()
    if exact.cofactor_det(ai) == 0:
        a[0, 0] += 1
        ai = a.astype(int).tolist()
    inv = exact.adjugate_inverse(ai)
    got = O.inverse(a)
    ref = np.array([[float(x) for x in row] for row in inv])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n,refl", [(16, 3), (100, 5)])
def test_inverse_closed_form_qd(n, refl):
    """A = Q D with Q orthogonal gives A^{-1} = D^{-2} A^T."""
    a, d, _ = synth.householder_qd(n, 5 * n, refl)
    ref = (a / d[None, :] ** 2).T
    np.testing.assert_allclose(O.inverse(a), ref, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(O.grad_logabsdet(a), a / d[None, :] ** 2,
                               rtol=1e-11, atol=1e-13)


def test_inverse_residual_and_singular():
    a = synth.normal(80, 1)
    inv = O.inverse(a)
    assert np.max(np.abs(a @ inv - np.eye(80))) < 1e-11
    z = a.copy()
    z[5] = 0
    with pytest.raises(np.linalg.LinAlgError):
        O.inverse(z)


def test_gradient_central_differences():
    """d log|det A| / dA_ij against central differences (h = 1e-6)."""
    a = synth.wishart(12, 8)
    g = O.grad_logabsdet(a)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(16):
        i, j = rng.integers(0, 12, 2)
        e = np.zeros_like(a)
        e[i, j] = h
        fd = (O.slogdet(a + e).logabsdet - O.slogdet(a - e).logabsdet) / (2 * h)
        assert abs(fd - g[i, j]) < 1e-7
