"""Batched factor and batched backward calls (mc_logdet_batched_factor,
mc_logdet_batched_backward) through the C ABI.

* The batched factor call gives the same (sign, log|det|, info) as the
  batched log-det call (same kernel, bit for bit), and factors with
  A[:, perm] = L U to rounding, and perm a permutation.
* The batched backward, run on those factors (and on single-matrix
  mc_logdet_factor factors), equals g_k * A_k^{-T} from the oracle's
  Gauss-Jordan inverse: FP64 within 1e-10 relative Frobenius, FP32 within
  1e-3 (the FP32 bar); member by member, with uneven sizes that span
  several 64-column blocks and ragged tails, and per-member g_k.
* Members whose forward failed (singular) get an all-NaN gradient; the
  others in the same launch are unaffected.
"""

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
SIZES = [1, 2, 17, 63, 64, 65, 130, 200, 257, 400]


def _mats(sizes, seed, dt):
    g = np.random.default_rng(seed)
    out = []
    for n in sizes:
        a = synth.wishart_from(g, n) if n > 8 else g.standard_normal((n, n)) + 3 * np.eye(n)
        out.append(a)
    return out, [torch.from_numpy(a).to(DEV, dt) for a in out]


def _relfro(x, ref):
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.mark.parametrize("dt,update", [(torch.float64, "native"), (torch.float32, "f32")])
def test_batched_factor_matches_batched_logdet(dt, update):
    print(f"[bgrad] factor {dt} {update}", flush=True)
    host, mats = _mats(SIZES, 3, dt)
    lus, perms, res = mc.factor_batched(mats, update=update)
    got = mc.read_result(res)
    ref = mc.logdet_batched(mats, update=update)
    for k, (a, lu, p) in enumerate(zip(host, lus, perms)):
        n = a.shape[0]
        assert got[k] == ref[k], (k, got[k], ref[k])
        pn = p.cpu().numpy()
        assert sorted(pn.tolist()) == list(range(n))
        f = lu.double().cpu().numpy()
        L = np.tril(f)
        U = np.triu(f, 1) + np.eye(n)
        a_in = mats[k].double().cpu().numpy()
        err = np.abs(a_in[:, pn] - L @ U).max()
        tol = (1e-11 if dt == torch.float64 else 1e-4) * n * max(1.0, np.abs(a_in).max())
        assert err <= tol, (k, n, err)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_batched_backward_against_oracle_inverse(dt):
    print(f"[bgrad] backward {dt}", flush=True)
    host, mats = _mats(SIZES, 4, dt)
    lus, perms, res = mc.factor_batched(mats)
    g = torch.tensor([0.5 + k for k in range(len(mats))], dtype=torch.float64, device=DEV)
    grads = mc.backward_batched(lus, perms, grad_out=g, fwd=res)
    bar = 1e-10 if dt == torch.float64 else 1e-3
    for k, (m, gr) in enumerate(zip(mats, grads)):
        a = m.double().cpu().numpy()
        ref = (0.5 + k) * O.grad_logabsdet(a)
        err = _relfro(gr.double().cpu().numpy(), ref)
        assert err <= bar, (k, a.shape[0], err)


def test_batched_backward_on_single_factors_and_large():
    """Factors from the single-matrix factor call (the blocked path), sizes
    up to 1100 (many column blocks), against the single-matrix backward."""
    sizes = [700, 1100, 129]
    host, mats = _mats(sizes, 5, torch.float64)
    lus, perms, fwds = [], [], []
    for m in mats:
        lu, p, r = mc.factor(m)
        lus.append(lu)
        perms.append(p)
        fwds.append(r)
    fwd = torch.cat(fwds)
    grads = mc.backward_batched(lus, perms, fwd=fwd)
    for k, (lu, p, r, gr) in enumerate(zip(lus, perms, fwds, grads)):
        single = mc.backward(lu, p, fwd=r)
        err = _relfro(gr.cpu().numpy(), single.cpu().numpy())
        assert err <= 1e-12, (k, err)
        ref = O.grad_logabsdet(host[k])
        assert _relfro(gr.cpu().numpy(), ref) <= 1e-10


def test_batched_backward_failed_member_is_nan():
    host, mats = _mats([50, 80, 120], 6, torch.float64)
    mats[1] = torch.zeros((80, 80), dtype=torch.float64, device=DEV)
    mats[1][:, :40] = torch.from_numpy(host[1][:, :40]).to(DEV)  # rank 40
    lus, perms, res = mc.factor_batched(mats)
    r = mc.read_result(res)
    assert r[1].info > 0 and r[0].info == 0 and r[2].info == 0
    grads = mc.backward_batched(lus, perms, fwd=res)
    assert torch.isnan(grads[1]).all()
    for k in (0, 2):
        ref = O.grad_logabsdet(host[k])
        assert _relfro(grads[k].cpu().numpy(), ref) <= 1e-10


def test_batched_backward_empty_and_argument_checks():
    import ctypes
    lib = mc.lib()
    fake = ctypes.c_void_p(256)
    assert lib.mc_logdet_batched_backward(fake, fake, fake, fake, 0, 10, 0, None,
                                          None, fake, fake, fake, 1 << 20, None) == 0
    assert lib.mc_logdet_batched_backward(fake, fake, fake, fake, -1, 10, 0, None,
                                          None, fake, fake, fake, 1 << 20, None) == -5
    assert lib.mc_logdet_batched_backward(fake, fake, fake, fake, 2, 20000, 0, None,
                                          None, fake, fake, fake, 1 << 20, None) == -6
    assert lib.mc_logdet_batched_backward(fake, fake, fake, fake, 2, 10, 0, None,
                                          None, fake, fake, fake, 8, None) == -100
