"""MI355X (gfx950) matrix-condensation log-determinant engine.

A thin ctypes binding over the C ABI in ``include/mc.h`` (``libmc.so``,
built in-tree by ``paper_1811_08057_amd.build``).  Every step of the
computation runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch supplies device memory (inputs, workspace, results) and
the current HIP stream.

Method: Dong, Barnett, Dhall, arXiv 1811.08057 -- repeated condensation
(Eqs. 1-3) with the pivot column of largest |a_kl| in each pivot row
(Section 2.2) and the pivot factored out of its row (Section 2.3).
"""

from __future__ import annotations

import ctypes
import os
from typing import NamedTuple, Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmc.so")

DTYPE_F64, DTYPE_F32 = 0, 1
UPDATE_NATIVE, UPDATE_F32, UPDATE_BF16X3 = 0, 1, 2
INFO_NONFINITE = -1

_UPDATES = {"native": UPDATE_NATIVE, "f32": UPDATE_F32,
            "bf16x3": UPDATE_BF16X3}

# Every symbol include/mc.h declares (checked by the test suite).
EXPORTS = ("mc_version", "mc_status_string", "mc_logdet_workspace",
           "mc_logdet", "mc_profile_enable", "mc_profile_read")


class MCError(RuntimeError):
    """A negative status from the C ABI."""


class Result(NamedTuple):
    sign: float
    logabsdet: float
    info: int


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_1811_08057_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    L.mc_version.restype = ctypes.c_int
    L.mc_status_string.argtypes = [ctypes.c_int]
    L.mc_status_string.restype = ctypes.c_char_p
    L.mc_logdet_workspace.argtypes = [i64, ctypes.c_int, ctypes.c_int, i64]
    L.mc_logdet_workspace.restype = sz
    L.mc_logdet.argtypes = [vp, i64, i64, ctypes.c_int, ctypes.c_int, i64, vp,
                            vp, sz, vp]
    L.mc_logdet.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    L.mc_profile_enable.argtypes = [ctypes.c_int]
    L.mc_profile_enable.restype = ctypes.c_int
    L.mc_profile_read.argtypes = [dp, ctypes.POINTER(ctypes.c_int64), dp, dp]
    L.mc_profile_read.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, what: str) -> None:
    if status != 0:
        msg = lib().mc_status_string(status).decode()
        raise MCError(f"{what}: status {status} ({msg})")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return DTYPE_F64
    if t.dtype == torch.float32:
        return DTYPE_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _update_code(update) -> int:
    if isinstance(update, str):
        return _UPDATES[update]
    return int(update)


def _square_rows(a: torch.Tensor) -> int:
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("expected a square matrix")
    if not a.is_cuda:
        raise ValueError("expected a device tensor")
    if a.shape[0] > 1 and a.stride(1) != 1:
        raise ValueError("rows must be contiguous (row-major, stride(1) == 1)")
    return max(a.stride(0), a.shape[0], 1)


def _stream_ptr(stream: Optional[torch.cuda.Stream], dev) -> int:
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    return s.cuda_stream


def workspace_bytes(n: int, dtype=torch.float64, update="native",
                    b: int = 0) -> int:
    code = DTYPE_F64 if dtype == torch.float64 else DTYPE_F32
    nb = lib().mc_logdet_workspace(n, code, _update_code(update), b)
    if nb == 0 and n >= 0:
        raise MCError("unsupported combination for the workspace query")
    return int(nb)


def new_workspace(n: int, device, dtype=torch.float64, update="native",
                  b: int = 0) -> torch.Tensor:
    return torch.empty(workspace_bytes(n, dtype, update, b), dtype=torch.uint8,
                       device=device)


def new_result(device, count: int = 1) -> torch.Tensor:
    """Device buffer for `count` mc_result structs (3 x 8 bytes each)."""
    return torch.empty((count, 3), dtype=torch.float64, device=device)


def logdet_async(a: torch.Tensor, result: torch.Tensor,
                 work: torch.Tensor, b: int = 0, update="native",
                 stream: Optional[torch.cuda.Stream] = None) -> None:
    """Enqueue mc_logdet on the stream; `result` receives the mc_result."""
    n = a.shape[0]
    lda = _square_rows(a)
    st = lib().mc_logdet(a.data_ptr(), n, lda, _dtype_code(a),
                         _update_code(update), b, result.data_ptr(),
                         work.data_ptr(), work.numel(),
                         _stream_ptr(stream, a.device))
    _check(st, "mc_logdet")


def read_result(result: torch.Tensor) -> list:
    """Copy mc_result structs to the host (synchronises)."""
    host = result.detach().cpu().contiguous()
    vals = host.numpy().reshape(-1, 3)
    infos = host.numpy().reshape(-1, 3).view("int64")[:, 2]
    return [Result(float(v[1]), float(v[0]), int(i))
            for v, i in zip(vals, infos)]


def slogdet(a: torch.Tensor, b: int = 0, update="native") -> Result:
    """(sign, log|det A|, info) of a square device matrix (synchronises)."""
    result = new_result(a.device)
    work = new_workspace(a.shape[0], a.device, a.dtype, update, b)
    logdet_async(a, result, work, b=b, update=update)
    return read_result(result)[0]


class Profile(NamedTuple):
    elapsed_ms: float
    launches: int
    alg_bytes: float
    alg_flops: float


def profile_enable(on: bool = True) -> None:
    """Start (resetting) or stop event timing of the dominant kernel."""
    _check(lib().mc_profile_enable(1 if on else 0), "mc_profile_enable")


def profile_read() -> Profile:
    ms, la = ctypes.c_double(), ctypes.c_int64()
    by, fl = ctypes.c_double(), ctypes.c_double()
    _check(lib().mc_profile_read(ctypes.byref(ms), ctypes.byref(la),
                                 ctypes.byref(by), ctypes.byref(fl)),
           "mc_profile_read")
    return Profile(ms.value, la.value, by.value, fl.value)
