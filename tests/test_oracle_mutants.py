"""Planted mistakes: each mutant of the oracle source must fail the pins.

Every case below rewrites one line of ``oracle/mc_oracle.c`` into a
plausible mistake (a dropped term, a wrong sign, a wrong index, the garbled
reading of Figure 6 step 4.1), builds the mutant into a temporary
directory on the CPU, and runs a short battery of exact and closed-form
checks against it.  A mutant that passes the battery would mean the pins
cannot tell that mistake from the paper's method.
"""

import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import exact

SRC = os.path.join(os.path.dirname(O.__file__), "mc_oracle.c")

MUTANTS = {
    "no_slot_move": ("wi[l] = wi[m - 1];", "(void)0;"),
    "no_pivot_row_slot_move": ("r[l] = r[m - 1];", "(void)0;"),
    "update_sign": ("wi[j] = wi[j] - prod;", "wi[j] = wi[j] + prod;"),
    "pivot_is_abs": ("const double p = row[l];",
                     "const double p = fabs(row[l]);"),
    "no_negative_count": ("if (p < 0.0) ++negatives;", "(void)0;"),
    "no_column_parity": ("sg *= perm_sign(piv_col, n);", "(void)0;"),
    "no_row_parity": ("sg *= perm_sign(piv_row, n);", "(void)0;"),
    "tie_largest_column": (
        "(key == bestkey && colid[j] < colid[best])) {\n                best = j;\n                bestkey = key;\n            }\n        } else if (rule == MCO_COL_FIRST_NONZERO)",
        "(key == bestkey && colid[j] > colid[best])) {\n                best = j;\n                bestkey = key;\n            }\n        } else if (rule == MCO_COL_FIRST_NONZERO)"),
    "signed_argmax": ("double a = fabs(row[j]);", "double a = row[j];"),
    "no_colid_update": ("colid[l] = colid[m - 1];", "(void)0;"),
    "eq2_case2_index": ("v = det2(akl, akj(j + 1), a(i, l), a(i, j + 1));",
                        "v = det2(akl, akj(j), a(i, l), a(i, j + 1));"),
    "eq2_case1_operands": ("v = det2(a(i, j), a(i, l), akj(j), akl);",
                           "v = det2(a(i, l), a(i, j), akj(j), akl);"),
    "eq2_case4_row": ("v = det2(akl, akj(j + 1), a(i + 1, l), a(i + 1, j + 1));",
                      "v = det2(akl, akj(j + 1), a(i, l), a(i + 1, j + 1));"),
    "singular_info": ("out->info = bad_step + 1;", "out->info = bad_step;"),
    "stash_after_move": ("const double c = wi[l];\n            wi[l] = wi[m - 1];",
                         "wi[l] = wi[m - 1];\n            const double c = wi[l];"),
    "inverse_update_sign": ("M[i * w + j] = M[i * w + j] - prod;",
                            "M[i * w + j] = M[i * w + j] + prod;"),
    "log_not_abs_sum": ("neumaier_add(&logsum, log(fabs(p)));",
                        "neumaier_add(&logsum, log(fabs(p)) * 0.5);"),
    # the compensation dropped: a plain running sum (Figure 6 step 4.4 as
    # printed), which the cancelling-diagonal pin must tell apart
    "plain_log_sum": ("static void neumaier_add(neumaier* a, double x)\n{",
                      "static void neumaier_add(neumaier* a, double x)\n{\n"
                      "    a->sum += x;\n    return;"),
    # ties to the smallest current slot instead of the smallest original
    # column: the same at step 0, different once slots have moved
    "tie_smallest_slot": (
        "(key == bestkey && colid[j] < colid[best])) {\n                best = j;\n                bestkey = key;\n            }\n        } else if (rule == MCO_COL_FIRST_NONZERO)",
        "(key == bestkey && j < best)) {\n                best = j;\n                bestkey = key;\n            }\n        } else if (rule == MCO_COL_FIRST_NONZERO)"),
}


def _battery():
    """Short pin battery; returns the list of failed checks."""
    failed = []

    def check(name, ok):
        if not ok:
            failed.append(name)

    def rel(a, b):
        return abs(a - b) / max(abs(b), 1.0)

    # exact integer determinants (Laplace)
    for n in [2, 3, 4, 5, 6]:
        for seed in range(4):
            a = synth.int_matrix(n, 1000 * n + seed)
            d = exact.cofactor_det(a.astype(int).tolist())
            if d == 0:
                continue
            r = O.slogdet(a)
            check(f"cofactor{n}.{seed}",
                  r.sign == (1 if d > 0 else -1)
                  and rel(r.logabsdet, math.log(abs(d))) < 1e-12)
    # closed form with a known sign: Q diag(d)
    a, d, refl = synth.householder_qd(30, 5, 3)
    r = O.slogdet(a)
    check("householder", r.sign == (-1) ** refl * np.prod(np.sign(d))
          and rel(r.logabsdet, float(np.sum(np.log(np.abs(d))))) < 1e-12)
    # pivot-row independence
    a = synth.uniform(16, 3)
    ref = O.slogdet(a)
    r2 = O.slogdet(a, rows=O.ROWS_FIG6, n_virt=4)
    check("row_order", r2.sign == ref.sign
          and rel(r2.logabsdet, ref.logabsdet) < 1e-12)
    a6 = synth.int_matrix(6, 6006)
    d6 = exact.cofactor_det(a6.astype(int).tolist())
    r6 = O.slogdet(a6, rows=O.ROWS_BOTTOM_UP)  # reversal of 6 rows is odd
    check("bottom_up", d6 != 0 and r6.sign == (1 if d6 > 0 else -1))
    # Eq. 2 one-step identity, exact integers, every pivot
    a = synth.int_matrix(4, 304)
    ai = a.astype(int).tolist()
    da = exact.cofactor_det(ai)
    ok = True
    for k in range(4):
        for l in range(4):
            if ai[k][l] == 0:
                continue
            b = O.condense_step(a, k, l)
            db = exact.cofactor_det([[int(round(x)) for x in rr] for rr in b])
            ok &= db == (-1) ** (k + l) * da * ai[k][l] ** 2
    check("eq2", ok)
    # tie break (smallest original column)
    t = np.array([[3.0, -3.0, 1.0, 3.0], [1.0, 2.0, 0.5, 0.25],
                  [0.0, 1.0, 4.0, 1.0], [2.0, 0.0, 1.0, 5.0]])
    check("tie", O.slogdet(t, pivots=True).piv_col[0] == 0)
    # singular row at step 3 -> info 4
    z = synth.uniform(7, 1)
    z[3] = 0
    check("singular", O.slogdet(z).info == 4)
    # pivot sequence on exact ties: the exact characterisation of the rule
    for seed in range(3):
        u = synth.unimodular_ties(20, 50 + seed)
        cols = [int(c) for c in O.slogdet(u, pivots=True).piv_col]
        check(f"unimodular_rule.{seed}",
              exact.satisfies_maxabs_rule(u.astype(int).tolist(), cols))
    # compensated log sum on a cancelling diagonal
    from tests.test_oracle_pivots import cancelling_diagonal
    cd, dd = cancelling_diagonal()
    want = math.fsum(math.log(abs(x)) for x in dd)
    check("compensated_sum", abs(O.slogdet(cd).logabsdet - want) <= 4e-16 * max(1.0, abs(want)))
    # explicit inverse vs closed form
    a, d, _ = synth.householder_qd(12, 7, 2)
    check("inverse", np.allclose(O.inverse(a), (a / d[None, :] ** 2).T,
                                 rtol=1e-10, atol=1e-12))
    return failed


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_battery_passes_on_the_oracle():
    assert _battery() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not unique"
    (tmp_path / "mc_oracle.h").write_text(
        open(SRC.replace(".c", ".h")).read())
    src = tmp_path / "mc_oracle.c"
    src.write_text(source.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", *O.CFLAGS, "-o", str(so), str(src), "-lm"])
    monkeypatch.setattr(O, "_LIB", str(so))
    monkeypatch.setattr(O, "_lib", None)
    failed = _battery()
    monkeypatch.setattr(O, "_lib", None)
    assert failed, f"mutant {name} passed every pin"
