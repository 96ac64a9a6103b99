"""mc_logdet_noalloc (the entry point that allocates nothing) against
mc_logdet on the same inputs, through the C ABI.

Two calls in a row on the library's fixed scratch array, the second with a
smaller matrix (so a stale workspace from the first would show), on the
plain path and the blocked path in FP64, FP32 and split-BF16x3; each result
must equal mc_logdet's (run with lookahead off, the schedule the no-alloc
call takes) and meet the FP64 oracle's bar: sign exact, log|det| within
1e-9 relative (FP64) or 1e-5 of the oracle on the FP32-rounded input.
Sizes above the array's capacity are refused before any launch.
"""

import ctypes

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
NOALLOC_BYTES = 40 * 1024 * 1024
TOO_LARGE = -103

CASES = [  # (dtype, update, b, first n, second n)
    (torch.float64, "native", 0, 1500, 700),
    (torch.float64, "native", 128, 2048, 1100),
    (torch.float64, "native", 64, 900, 333),
    (torch.float32, "f32", 128, 2048, 1500),
    (torch.float32, "bf16x3", 64, 1300, 257),
]


def _noalloc(a, update, b, out):
    lib = mc.lib()
    st = lib.mc_logdet_noalloc(
        ctypes.c_void_p(a.data_ptr()), ctypes.c_int64(a.shape[0]),
        ctypes.c_int64(a.stride(0)), ctypes.c_int(mc._dtype_code(a)),
        ctypes.c_int(mc._update_code(update)), ctypes.c_int64(b),
        ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    return st


def _reference(a, update, b):
    old = mc.lookahead_enable(False)
    try:
        return mc.slogdet(a, b=b, update=update)
    finally:
        mc.lookahead_enable(old)


@pytest.mark.parametrize("dt,update,b,n1,n2", CASES)
def test_noalloc_matches_logdet_twice(dt, update, b, n1, n2):
    mc.lib().mc_logdet_noalloc.restype = ctypes.c_int
    out = mc.new_result(DEV)  # allocated before the calls
    for n, seed in ((n1, 11), (n2, 12)):
        print(f"[noalloc] {dt} {update} b={b} n={n}", flush=True)
        a_np = synth.normal(n, seed + n)
        a = torch.from_numpy(a_np).to(DEV, dt)
        assert _noalloc(a, update, b, out) == 0
        got = mc.read_result(out)[0]
        ref = _reference(a, update, b)
        assert got.info == ref.info == 0
        assert got.sign == ref.sign
        assert abs(got.logabsdet - ref.logabsdet) <= 1e-12 * max(1.0, abs(ref.logabsdet))
        o = O.slogdet(a.cpu().double().numpy())
        tol = 1e-9 if dt == torch.float64 else 1e-5
        assert got.sign == o.sign
        assert abs(got.logabsdet - o.logabsdet) <= tol * max(1.0, abs(o.logabsdet))


def test_noalloc_refuses_too_large_and_bad_args():
    lib = mc.lib()
    lib.mc_logdet_noalloc.restype = ctypes.c_int
    out = mc.new_result(DEV)
    n = 2600  # the FP64 blocked workspace exceeds the array
    assert lib.mc_logdet_workspace(n, 0, 0, -1) > NOALLOC_BYTES
    a = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    assert _noalloc(a, "native", -1, out) == TOO_LARGE
    assert b"scratch" in lib.mc_status_string(TOO_LARGE)
    small = torch.eye(4, dtype=torch.float64, device=DEV)
    st = lib.mc_logdet_noalloc(ctypes.c_void_p(small.data_ptr()), ctypes.c_int64(4),
                               ctypes.c_int64(3), 0, 0, ctypes.c_int64(0),
                               ctypes.c_void_p(out.data_ptr()), None)
    assert st == -3
    # n = 0 writes {0, +1, 0}
    z = torch.zeros((1, 1), dtype=torch.float64, device=DEV)
    st = lib.mc_logdet_noalloc(ctypes.c_void_p(z.data_ptr()), ctypes.c_int64(0),
                               ctypes.c_int64(1), 0, 0, ctypes.c_int64(0),
                               ctypes.c_void_p(out.data_ptr()), None)
    assert st == 0
    torch.cuda.synchronize()
    r = mc.read_result(out)[0]
    assert (r.sign, r.logabsdet, r.info) == (1.0, 0.0, 0)
