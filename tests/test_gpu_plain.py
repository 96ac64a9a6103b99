"""GPU parity of the plain (unblocked) FP64 condensation path.

Every case runs the HIP path through the C ABI and compares with the FP64
CPU oracle on the same seeded input: sign exact, log|det| within 1e-9
relative (|d| <= 1e-9 * max(|ref|, 1)), info equal.
"""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_08057_amd as mc  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-9
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run(a_np, b=0, update="native", dtype=torch.float64):
    print(f"[plain] n={a_np.shape[0]} b={b} update={update}", flush=True)
    a = torch.from_numpy(np.ascontiguousarray(a_np)).to(DEV, dtype)
    r = mc.slogdet(a, b=b, update=update)
    return r


def assert_parity(got, ref, tol=TOL):
    assert got.info == ref.info, (got, ref)
    assert got.sign == ref.sign, (got, ref)
    if math.isfinite(ref.logabsdet):
        assert abs(got.logabsdet - ref.logabsdet) <= tol * max(
            abs(ref.logabsdet), 1.0), (got, ref)
    else:
        assert (math.isnan(got.logabsdet) and math.isnan(ref.logabsdet)) or \
            got.logabsdet == ref.logabsdet


SIZES = [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127,
         128, 129, 255, 256, 257, 300, 511, 513]


@pytest.mark.parametrize("n", SIZES)
def test_plain_random_sizes(n):
    for a in (synth.uniform(n, 100 + n), synth.normal(n, 200 + n)):
        assert_parity(run(a), O.slogdet(a))


def test_plain_integer_ties():
    """Integer entries in [-2, 2]: many exact ties in the pivot search."""
    for seed in range(40):
        n = 3 + seed % 30
        a = synth.int_matrix(n, 5000 + seed, lo=-2, hi=2)
        ref = O.slogdet(a)
        if ref.info != 0 or ref.logabsdet < -20:
            continue  # singular in exact arithmetic
        assert_parity(run(a), ref)


def test_plain_uniform_n1000_expected():
    """The N = 1000 U[-1, 1] workload (seed 1), against the stored oracle
    value and a live oracle run."""
    a = synth.make("uniform_n1000")
    ref = O.slogdet(a)
    with open(os.path.join(GOLDEN, "expected_uniform_n1000.json")) as f:
        stored = json.load(f)["f64"]
    assert stored["sign"] == ref.sign and stored["logabsdet"] == ref.logabsdet
    assert_parity(run(a), ref)


@pytest.mark.parametrize("n,refl", [(1024, 5), (2048, 9)])
def test_plain_closed_form_qd(n, refl):
    a, d, r_ = synth.householder_qd(n, 17 * n, refl)
    got = run(a)
    assert got.info == 0
    assert got.sign == (-1) ** r_ * np.prod(np.sign(d))
    ref = float(np.sum(np.log(np.abs(d))))
    assert abs(got.logabsdet - ref) <= TOL * max(abs(ref), 1.0)


def test_plain_n0_and_singular_and_nonfinite():
    assert run(np.zeros((0, 0))) == mc.Result(1.0, 0.0, 0)
    a = synth.uniform(50, 3)
    z = a.copy()
    z[17] = 0.0
    assert_parity(run(z), O.slogdet(z))
    zc = a.copy()
    zc[:, 5] = 0.0
    assert_parity(run(zc), O.slogdet(zc))
    r = run(np.zeros((5, 5)))
    assert (r.sign, r.logabsdet, r.info) == (0.0, -math.inf, 1)
    for bad in [np.nan, np.inf]:
        for pos in [(0, 3), (20, 20), (49, 0)]:
            b = a.copy()
            b[pos] = bad
            got = run(b)
            assert got.info == mc.INFO_NONFINITE and got.sign == 0
            assert math.isnan(got.logabsdet)
    r = run(np.array([[0.0]]))
    assert r.info == 1 and r.sign == 0


def test_plain_strided_rows():
    n, lda = 77, 101
    a = synth.normal(n, 9)
    big = torch.full((n, lda), float("nan"), dtype=torch.float64, device=DEV)
    big[:, :n] = torch.from_numpy(a).to(DEV)
    view = big[:, :n]
    assert view.stride(0) == lda
    got = mc.slogdet(view)
    assert_parity(got, O.slogdet(a))


def test_plain_deterministic_and_input_untouched():
    a_np = synth.normal(700, 44)
    a = torch.from_numpy(a_np).to(DEV)
    before = a.clone()
    r1 = mc.slogdet(a)
    r2 = mc.slogdet(a)
    assert r1 == r2  # bitwise
    assert torch.equal(a, before)


def test_plain_reused_workspace_stream_ordered():
    """One workspace, several matrices back to back on one stream."""
    n = 300
    work = mc.new_workspace(n, DEV)
    res = mc.new_result(DEV, 4)
    mats = [synth.uniform(n, 900 + k) for k in range(4)]
    for k, m in enumerate(mats):
        mc.logdet_async(torch.from_numpy(m).to(DEV), res[k], work)
    for got, m in zip(mc.read_result(res), mats):
        assert_parity(got, O.slogdet(m))


def test_plain_normal_n8000_expected():
    """Full size (N = 8000, N(0,1), seed 2) against the stored oracle value
    written by tests/golden/make_expected.py."""
    path = os.path.join(GOLDEN, "expected_normal_n8000.json")
    if not os.path.exists(path):
        pytest.skip("expected value not generated")
    with open(path) as f:
        e = json.load(f)["f64"]
    ref = O.SlogdetResult(e["sign"], e["logabsdet"], e["info"])
    assert_parity(run(synth.make("normal_n8000")), ref)
