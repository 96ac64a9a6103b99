"""Python access to the plain FP64 CPU oracle (``oracle/mc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the reference the GPU engine is
checked against; only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
engine (``paper_1811_08057_amd``) and never imports it.

Functions follow arXiv 1811.08057: ``slogdet`` is the condensation loop of
Figure 6 with one process (Eqs. 1-3, Sections 2.2-2.4); ``condense_step`` is
one application of Eq. 2 (or Eq. 3 with the pivot factored out of row k);
``inverse`` is a separate Gauss-Jordan elimination used to check gradients.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.c")
_LIB = os.path.join(_HERE, "libmc_oracle.so")

ROWS_TOP_DOWN, ROWS_BOTTOM_UP, ROWS_EXPLICIT, ROWS_FIG6 = 0, 1, 2, 3
COL_MAXABS, COL_FIRST_NONZERO, COL_CLOSEST_TO_ONE = 0, 1, 2
INFO_NONFINITE = -1
INFO_PARTIAL = -2

# Plain build: contraction off so products and differences round separately.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-fopenmp", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/libmc_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [("logabsdet", ctypes.c_double), ("sign", ctypes.c_double),
                ("info", ctypes.c_int64)]


class SlogdetResult(NamedTuple):
    sign: float
    logabsdet: float
    info: int
    piv_row: Optional[np.ndarray] = None
    piv_col: Optional[np.ndarray] = None
    piv_val: Optional[np.ndarray] = None


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.mco_slogdet.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int, i64p, ctypes.c_int64,
                                  ctypes.c_int, ctypes.POINTER(_Result),
                                  i32p, i32p, dp]
        L.mco_slogdet.restype = ctypes.c_int
        L.mco_slogdet_steps.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64,
                                        ctypes.POINTER(_Result)]
        L.mco_slogdet_steps.restype = ctypes.c_int
        L.mco_condense_step.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int, dp]
        L.mco_condense_step.restype = ctypes.c_int
        L.mco_inverse.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, dp,
                                  ctypes.c_int64]
        L.mco_inverse.restype = ctypes.c_int
        L.mco_slogdet_gaps.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.POINTER(_Result), i32p, dp]
        L.mco_slogdet_gaps.restype = ctypes.c_int
        L.mco_set_threads.argtypes = [ctypes.c_int]
        L.mco_set_threads.restype = ctypes.c_int
        L.mco_num_procs.restype = ctypes.c_int
        _lib = L
    return _lib


def _as_f64(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("expected a square matrix")
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def slogdet(a: np.ndarray, rows: int = ROWS_TOP_DOWN,
            row_order: Optional[Sequence[int]] = None, n_virt: int = 0,
            col_rule: int = COL_MAXABS, pivots: bool = False) -> SlogdetResult:
    """(sign, log|det A|, info) by condensation.  FP32 input is widened to
    FP64 first, so an FP32 matrix is judged on its own rounded values."""
    a = _as_f64(a)
    n = a.shape[0]
    order = None
    if row_order is not None:
        order = np.ascontiguousarray(row_order, dtype=np.int64)
        if order.shape != (n,):
            raise ValueError("row_order must have n entries")
    pr = np.zeros(max(n, 1), np.int32) if pivots else None
    pc = np.zeros(max(n, 1), np.int32) if pivots else None
    pv = np.zeros(max(n, 1), np.float64) if pivots else None
    res = _Result()
    rc = lib().mco_slogdet(_ptr(a, ctypes.c_double), n, max(n, 1), rows,
                           _ptr(order, ctypes.c_int64), n_virt, col_rule,
                           ctypes.byref(res), _ptr(pr, ctypes.c_int32),
                           _ptr(pc, ctypes.c_int32), _ptr(pv, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"mco_slogdet rejected its arguments ({rc})")
    if pivots:
        return SlogdetResult(res.sign, res.logabsdet, res.info, pr[:n], pc[:n],
                             pv[:n])
    return SlogdetResult(res.sign, res.logabsdet, res.info)


def slogdet_gaps(a: np.ndarray):
    """(SlogdetResult with piv_col, gaps): the top-down, largest-|a| run with
    each step's relative margin of the pivot over the runner-up in its row
    (0 = a tie the tie rule decided, 1 = a single active slot)."""
    a = _as_f64(a)
    n = a.shape[0]
    pc = np.zeros(max(n, 1), np.int32)
    gap = np.full(max(n, 1), np.nan)
    res = _Result()
    rc = lib().mco_slogdet_gaps(_ptr(a, ctypes.c_double), n, max(n, 1),
                                ctypes.byref(res), _ptr(pc, ctypes.c_int32),
                                _ptr(gap, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"mco_slogdet_gaps rejected its arguments ({rc})")
    return SlogdetResult(res.sign, res.logabsdet, res.info, None, pc[:n]), gap[:n]


def set_threads(threads: int) -> int:
    """OpenMP threads for the row updates of each step; returns the previous
    count.  The results do not depend on it."""
    return int(lib().mco_set_threads(int(threads)))


def num_procs() -> int:
    return int(lib().mco_num_procs())


def slogdet_steps(a: np.ndarray, max_steps: int) -> SlogdetResult:
    """The first ``max_steps`` condensation steps only (timing samples)."""
    a = _as_f64(a)
    n = a.shape[0]
    res = _Result()
    rc = lib().mco_slogdet_steps(_ptr(a, ctypes.c_double), n, max(n, 1),
                                 max_steps, ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"mco_slogdet_steps rejected its arguments ({rc})")
    return SlogdetResult(res.sign, res.logabsdet, res.info)


def condense_step(a: np.ndarray, k: int, l: int, factored: bool = False
                  ) -> np.ndarray:
    """B from Eq. 2 (or B* from Eq. 3 when ``factored``) for pivot (k, l)."""
    a = _as_f64(a)
    n = a.shape[0]
    b = np.empty((n - 1, n - 1), np.float64)
    rc = lib().mco_condense_step(_ptr(a, ctypes.c_double), n, n, k, l,
                                 int(factored), _ptr(b, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"mco_condense_step rejected its arguments ({rc})")
    return b


def inverse(a: np.ndarray) -> np.ndarray:
    """A^{-1} by Gauss-Jordan; raises on a singular matrix."""
    a = _as_f64(a)
    n = a.shape[0]
    out = np.empty((n, n), np.float64)
    rc = lib().mco_inverse(_ptr(a, ctypes.c_double), n, max(n, 1),
                           _ptr(out, ctypes.c_double), max(n, 1))
    if rc == 1:
        raise np.linalg.LinAlgError("singular matrix")
    if rc != 0:
        raise ValueError(f"mco_inverse rejected its arguments ({rc})")
    return out


def grad_logabsdet(a: np.ndarray) -> np.ndarray:
    """d log|det A| / dA = A^{-T}, from the explicit inverse."""
    return inverse(a).T.copy()
