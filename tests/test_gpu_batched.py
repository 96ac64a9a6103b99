"""GPU parity of the batched persistent path (many matrices, uneven sizes).

Every member is compared with the FP64 oracle on the same input (FP32
members: the oracle on the FP32-rounded input): FP64 sign exact and
log|det| within 1e-9 relative; FP32 / split-BF16x3 within 1e-5 relative.
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
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_08057_amd as mc  # noqa: E402

DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(got, ref):
    return abs(got.logabsdet - ref.logabsdet) / max(abs(ref.logabsdet), 1.0)


def check(got, ref, tol):
    assert got.info == ref.info, (got, ref)
    assert got.sign == ref.sign, (got, ref)
    if math.isfinite(ref.logabsdet):
        assert rel(got, ref) <= tol, (got, ref, rel(got, ref))


def to_dev(mats, dtype):
    return [torch.from_numpy(np.ascontiguousarray(m)).to(DEV, dtype)
            for m in mats]


# b = 100 and 128: panels of more than four 16-column blocks (the solve's
# wide form), 100 with a partial last block
@pytest.mark.parametrize("b", [-1, 16, 64, 100, 128])
def test_batched_f64_mixed_sizes(b):
    rng = np.random.default_rng(11)
    sizes = [1, 2, 3, 17, 64, 65, 100, 129, 200, 257, 300, 511] + \
        list(rng.integers(1, 400, 20))
    mats = [synth.normal(int(n), 1000 + i) for i, n in enumerate(sizes)]
    print(f"[batched] f64 b={b} sizes={sizes}", flush=True)
    got = mc.logdet_batched(to_dev(mats, torch.float64), b=b)
    for g, m in zip(got, mats):
        check(g, O.slogdet(m), 1e-9)


@pytest.mark.parametrize("b", [100, 128])
def test_batched_f32_wide_panels(b):
    g = synth.rng(23)
    sizes = [int(n) for n in g.integers(100, 600, 10)] + [129, 257]
    mats = [synth.wishart_from(g, n).astype(np.float32) for n in sizes]
    print(f"[batched] f32 b={b} sizes={sizes}", flush=True)
    got = mc.logdet_batched(to_dev(mats, torch.float32), b=b)
    for gg, m in zip(got, mats):
        check(gg, O.slogdet(m), 1e-5)


@pytest.mark.parametrize("update", ["native", "f32", "bf16x3"])
def test_batched_f32_wishart(update):
    g = synth.rng(21)
    sizes = [int(n) for n in g.integers(16, 700, 24)]
    mats = [synth.wishart_from(g, n).astype(np.float32) for n in sizes]
    print(f"[batched] f32 {update} sizes={sizes}", flush=True)
    got = mc.logdet_batched(to_dev(mats, torch.float32), update=update)
    worst = 0.0
    for gg, m in zip(got, mats):
        ref = O.slogdet(m)
        check(gg, ref, 1e-5)
        worst = max(worst, rel(gg, ref))
    print(f"[batched] f32 {update}: worst rel err {worst:.3e}")


def test_batched_special_members():
    a = synth.uniform(90, 2)
    z = a.copy()
    z[40] = 0.0
    nf = a.copy()
    nf[7, 7] = np.nan
    mats = [a, z, nf, np.zeros((0, 0)), synth.uniform(5, 3)]
    print("[batched] special members", flush=True)
    got = mc.logdet_batched(to_dev(mats, torch.float64), b=16)
    check(got[0], O.slogdet(a), 1e-9)
    check(got[1], O.slogdet(z), 1e-9)
    assert got[2].info == mc.INFO_NONFINITE and got[2].sign == 0
    assert got[3] == mc.Result(1.0, 0.0, 0)
    check(got[4], O.slogdet(mats[4]), 1e-9)


def test_batched_member_beyond_n_max_is_flagged():
    """A member larger than the declared n_max is refused on the device
    with MC_INFO_BADARG; the other members are unaffected."""
    mats = to_dev([synth.uniform(40, 1), synth.uniform(30, 2)], torch.float64)
    plan = mc.BatchedPlan(mats, b=16)
    # declare a smaller bound than the first member's size, same workspace
    plan.n_max = 35
    plan.run()
    got = plan.results()
    assert got[0].info == mc.INFO_BADARG and got[0].sign == 0
    check(got[1], O.slogdet(synth.uniform(30, 2)), 1e-9)


def test_batched_graph_replays():
    """Capture the batched call in a hipGraph; replay it several times with
    eager work and synchronisations between replays; every replay must give
    the eager result."""
    g = synth.rng(7)
    sizes = [int(n) for n in g.integers(20, 300, 40)]
    mats = [synth.wishart_from(g, n) for n in sizes]
    plan = mc.BatchedPlan(to_dev(mats, torch.float64))
    plan.run()
    eager = plan.results()
    for m, e in zip(mats, eager):
        check(e, O.slogdet(m), 1e-9)
    plan.capture()
    for rep in range(4):
        plan.result.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        assert plan.results() == eager, f"replay {rep}"


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batched_wishart_batch512_expected(precision):
    """The 512-matrix Wishart workload (sizes U{32..1024}, seed 4) against
    the stored oracle values of tests/golden/make_expected.py."""
    path = os.path.join(GOLDEN, "expected_wishart_batch512.json")
    with open(path) as f:
        exp = json.load(f)
    sizes, mats = synth.make("wishart_batch512")
    assert sizes == exp["sizes"]
    # the bytes the oracle values were computed on (exact Gram products)
    assert synth.sha256_of(mats) == exp["sha256_f64"]
    dtype = torch.float64 if precision == "f64" else torch.float32
    if precision == "f32":
        assert synth.sha256_of([m.astype(np.float32) for m in mats]) == exp["sha256_f32"]
    tol = 1e-9 if precision == "f64" else 1e-5
    print(f"[batched] wishart_batch512 {precision}", flush=True)
    for update in (["native"] if precision == "f64" else ["f32", "bf16x3"]):
        got = mc.logdet_batched(to_dev(mats, dtype), update=update)
        worst = 0.0
        for gg, e in zip(got, exp[precision]):
            ref = O.SlogdetResult(e["sign"], e["logabsdet"], e["info"])
            check(gg, ref, tol)
            worst = max(worst, rel(gg, ref))
        print(f"[batched] 512 {precision} {update}: worst {worst:.3e}")


def test_autotune_produces_valid_table():
    before = mc.tune_get(torch.float64)
    table = mc.autotune_batched(torch.float64, n_max=300)
    print(f"[batched] tuned table {table} (before {before})", flush=True)
    b, tile = table
    assert all(1 <= x <= 128 for x in b) and all(t in (32, 64) for t in tile)
    mats = [synth.normal(n, n) for n in (50, 150, 250)]
    got = mc.logdet_batched(to_dev(mats, torch.float64))
    for gg, m in zip(got, mats):
        check(gg, O.slogdet(m), 1e-9)
    mc.tune_set(*before, dtype=torch.float64)
    assert mc.tune_get(torch.float64) == before


def test_batched_plan_routes_large_members():
    """Members of at least blocked_min_n rows go through the blocked path,
    the rest through the batched launch: the results land in
    the members' own order and meet the FP64 bar of the oracle, as with
    every member in the batched launch; a captured replay gives the same."""
    sizes = [300, 1100, 64, 1024, 511]
    mats = [synth.normal(n, 4000 + i) for i, n in enumerate(sizes)]
    devs = to_dev(mats, torch.float64)
    plan = mc.BatchedPlan(devs, blocked_min_n=1024)
    assert plan.large == [1, 3] and plan.small == [0, 2, 4]
    plan.run()
    routed = plan.results()
    every = mc.BatchedPlan(devs, blocked_min_n=None)
    every.run()
    batched = every.results()
    for m, r, q in zip(mats, routed, batched):
        ref = O.slogdet(m)
        assert r.info == ref.info and r.sign == ref.sign
        assert q.info == ref.info and q.sign == ref.sign
        assert abs(r.logabsdet - ref.logabsdet) <= 1e-9 * max(1.0, abs(ref.logabsdet))
        assert abs(q.logabsdet - ref.logabsdet) <= 1e-9 * max(1.0, abs(ref.logabsdet))
    plan.capture()
    plan.result.fill_(float("nan"))
    plan.small_result.fill_(float("nan"))
    torch.cuda.synchronize()
    plan.replay()
    torch.cuda.synchronize()
    assert plan.results() == routed


def test_autotune_cached_stores_and_reuses(tmp_path):
    """autotune_cached: the first call tunes and stores the table, the second
    reads it back from the cache file; the table the library then holds is
    valid and the batched results are unchanged by it."""
    path = str(tmp_path / "tune.json")
    old = mc.tune_get(torch.float64)
    try:
        b1, t1, src1 = mc.autotune_cached(torch.float64, "native", 256, DEV, path)
        assert src1 == "tuned"
        b2, t2, src2 = mc.autotune_cached(torch.float64, "native", 256, DEV, path)
        assert (src2, b2, t2) == ("cache", b1, t1)
        assert all(1 <= b <= 128 for b in b2) and all(t in (32, 64) for t in t2)
        mats = [torch.from_numpy(synth.normal(n, 40 + n)).to(DEV) for n in (50, 120, 250)]
        got = mc.logdet_batched(mats)
        for m, g in zip(mats, got):
            ref = O.slogdet(m.cpu().numpy())
            assert g.sign == ref.sign
            assert abs(g.logabsdet - ref.logabsdet) <= 1e-9 * max(1.0, abs(ref.logabsdet))
    finally:
        mc.tune_set(*old, torch.float64)


def test_batched_plan_concurrent_equals_sequential():
    """The batch's small members beside its large ones (the batched launch on
    a second stream, off XCD 0) give the same bits as one after the other,
    eagerly and replayed from a graph."""
    g = np.random.default_rng(77)
    sizes = [1100, 40, 300, 1030, 700, 5, 1024, 999]
    mats = [torch.from_numpy(synth.wishart_from(g, n)).to(DEV) for n in sizes]
    seq = mc.BatchedPlan(mats, blocked_min_n=1024, concurrent=False)
    seq.run()
    ref = seq.results()
    con = mc.BatchedPlan(mats, blocked_min_n=1024)
    assert con.concurrent
    con.run()
    assert con.results() == ref
    con.capture()
    for _ in range(3):
        con.small_result.fill_(float("nan"))
        con.result.fill_(float("nan"))
        con.replay()
        torch.cuda.synchronize()
        assert con.results() == ref
    for m, r in zip(mats, ref):
        o = O.slogdet(m.cpu().numpy())
        assert r.sign == o.sign
        assert abs(r.logabsdet - o.logabsdet) <= 1e-9 * max(1.0, abs(o.logabsdet))
