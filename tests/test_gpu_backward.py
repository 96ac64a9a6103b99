"""GPU factor call and backward (d log|det A| / dA = A^{-T}).

The factors are checked by reconstruction (A[:, perm] = L U) and by the
log-determinant they imply; the gradient against the oracle's explicit
Gauss-Jordan inverse, the closed form A^{-T} = A D^{-2} for A = Q diag(d),
and central differences of the oracle's log|det| (h = 1e-6, FP64).
"""

import math

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_08057_amd as mc  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def rel_fro(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


@pytest.mark.parametrize("b", [16, 32, 64])
def test_factor_reconstructs(b):
    for n in [1, 2, 3, 17, 65, 129, 300, 513]:
        a = synth.normal(n, 40 + n)
        print(f"[factor] n={n} b={b}", flush=True)
        lu, perm, res = mc.factor(dev(a), b=b)
        r = mc.read_result(res)[0]
        ref = O.slogdet(a)
        assert r.sign == ref.sign and r.info == 0
        assert abs(r.logabsdet - ref.logabsdet) <= 1e-9 * max(1, abs(ref.logabsdet))
        lu = lu.cpu().numpy()
        p = perm.cpu().numpy()
        assert sorted(p.tolist()) == list(range(n))
        L = np.tril(lu)
        U = np.triu(lu, 1) + np.eye(n)
        err = np.max(np.abs(a[:, p] - L @ U))
        assert err <= 1e-11 * max(1.0, np.max(np.abs(a))) * n, (n, err)
        # the pivots are L's diagonal; their log sum is log|det|
        assert abs(np.sum(np.log(np.abs(np.diag(lu)))) - ref.logabsdet) <= \
            1e-9 * max(1, abs(ref.logabsdet))


@pytest.mark.parametrize("n", [1, 2, 5, 40, 64, 65, 130, 257])
def test_backward_vs_oracle_inverse(n):
    a = synth.wishart(n, 500 + n) + 0.1 * synth.normal(n, 600 + n)
    print(f"[backward] n={n}", flush=True)
    lu, perm, _ = mc.factor(dev(a), b=32)
    g = mc.backward(lu, perm).cpu().numpy()
    ref = O.grad_logabsdet(a)
    assert rel_fro(g, ref) <= 1e-10, rel_fro(g, ref)


def test_backward_scaled_by_grad_out():
    a = synth.normal(50, 3)
    lu, perm, _ = mc.factor(dev(a), b=16)
    g1 = mc.backward(lu, perm).cpu().numpy()
    g2 = mc.backward(lu, perm, torch.tensor(-2.5, dtype=torch.float64,
                                            device=DEV)).cpu().numpy()
    np.testing.assert_allclose(g2, -2.5 * g1, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,refl", [(1024, 7), (2048, 3)])
def test_backward_closed_form_qd(n, refl):
    a, d, _ = synth.householder_qd(n, 77 + n, refl)
    lu, perm, _ = mc.factor(dev(a), b=64)
    g = mc.backward(lu, perm).cpu().numpy()
    assert rel_fro(g, a / d[None, :] ** 2) <= 1e-11


def test_backward_central_differences():
    """Oracle log|det| at A +- h e_ij, h = 1e-6, against the GPU gradient
    (expected FD error ~ eps |f| / h ~ 1e-8)."""
    n = 48
    a = synth.wishart(n, 9)
    lu, perm, _ = mc.factor(dev(a), b=16)
    g = mc.backward(lu, perm).cpu().numpy()
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(16):
        i, j = rng.integers(0, n, 2)
        e = np.zeros_like(a)
        e[i, j] = h
        fd = (O.slogdet(a + e).logabsdet - O.slogdet(a - e).logabsdet) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6, (i, j, fd, g[i, j])
    # and along a random unit-Frobenius direction
    v = rng.standard_normal((n, n))
    v /= np.linalg.norm(v)
    fd = (O.slogdet(a + h * v).logabsdet - O.slogdet(a - h * v).logabsdet) / (2 * h)
    assert abs(fd - float(np.sum(g * v))) <= 1e-6


def test_backward_f32_wishart():
    n = 300
    a = synth.wishart(n, 12).astype(np.float32)
    lu, perm, _ = mc.factor(dev(a, torch.float32), b=32)
    g = mc.backward(lu, perm).cpu().numpy().astype(np.float64)
    err = rel_fro(g, O.grad_logabsdet(a))
    print(f"[backward] f32 rel Frobenius error {err:.3e}")
    assert err <= 1e-3


@pytest.mark.parametrize("budget", [None, 0])
def test_autograd_keep_and_recompute(budget):
    a_np = synth.wishart(120, 4) + 0.05 * synth.normal(120, 5)
    a = dev(a_np).requires_grad_(True)
    sign, logabs = mc.slogdet_autograd(a, b=32, mem_budget=budget)
    (3.0 * logabs).backward()
    ref = O.slogdet(a_np)
    assert float(sign) == ref.sign
    assert abs(float(logabs) - ref.logabsdet) <= 1e-9 * max(1, abs(ref.logabsdet))
    assert rel_fro(a.grad.cpu().numpy(), 3.0 * O.grad_logabsdet(a_np)) <= 1e-10


def test_factor_singular_reports_info():
    a = synth.uniform(40, 2)
    a[13] = 0.0
    _, _, res = mc.factor(dev(a), b=16)
    r = mc.read_result(res)[0]
    ref = O.slogdet(a)
    assert (r.sign, r.info) == (ref.sign, ref.info) and r.logabsdet == -math.inf


def test_backward_after_failed_forward_is_nan():
    """A singular or non-finite input: the forward reports it (info != 0)
    and the backward, given the forward's result, returns an all-NaN
    gradient instead of one built from invalid factors -- decided on the
    device (no host synchronisation in MCLogDet)."""
    a = synth.uniform(150, 4)
    z = a.copy()
    z[40] = 0.0
    nf = a.copy()
    nf[3, 7] = np.nan
    for m, info in ((z, 41), (nf, mc.INFO_NONFINITE)):
        x = dev(m).requires_grad_(True)
        sign, logabs = mc.slogdet_autograd(x, b=32)
        assert float(sign) == 0.0
        logabs.backward()
        assert torch.isnan(x.grad).all()
        lu, perm, res = mc.factor(dev(m), b=32)
        assert mc.read_result(res)[0].info == info
        g = mc.backward(lu, perm, fwd=res)
        assert torch.isnan(g).all()
    # a good factorisation with fwd given: an ordinary gradient
    lu, perm, res = mc.factor(dev(a), b=32)
    g = mc.backward(lu, perm, fwd=res).cpu().numpy()
    assert rel_fro(g, O.grad_logabsdet(a)) <= 1e-10


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_backward_recompute_matches_kept_factors(dtype):
    """mc_logdet_backward_recompute (factors rebuilt inside the library)
    against the backward on kept factors and the oracle's inverse; the
    autograd function takes that route under a memory budget."""
    n = 700
    a = synth.wishart(n, 71)
    x = dev(a, dtype)
    lu, perm, res = mc.factor(x, b=64)
    kept = mc.backward(lu, perm, fwd=res)
    out = mc.new_result(DEV)
    again = mc.backward_recompute(x, b=64, out=out)
    r = mc.read_result(out)[0]
    ref_r = mc.read_result(res)[0]
    assert r == ref_r
    # the same kernels on the same input: bitwise
    assert torch.equal(kept, again)
    tol = 1e-10 if dtype == torch.float64 else 1e-4
    a_in = a if dtype == torch.float64 else a.astype(np.float32).astype(np.float64)
    assert rel_fro(again.double().cpu().numpy(), O.grad_logabsdet(a_in)) <= tol
    y = x.clone().requires_grad_(True)
    _, logabs = mc.slogdet_autograd(y, b=64, mem_budget=0)
    logabs.backward()
    assert torch.equal(y.grad, kept)
