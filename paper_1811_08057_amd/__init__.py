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
PIVOT_MAXABS, PIVOT_FIRST_NONZERO, PIVOT_CLOSEST_TO_ONE = 0, 1, 2
_RULES = {"maxabs": PIVOT_MAXABS, "first_nonzero": PIVOT_FIRST_NONZERO,
          "closest_to_one": PIVOT_CLOSEST_TO_ONE}

_UPDATES = {"native": UPDATE_NATIVE, "f32": UPDATE_F32,
            "bf16x3": UPDATE_BF16X3}

# Every symbol include/mc.h declares (checked by the test suite).
EXPORTS = ("mc_version", "mc_status_string", "mc_logdet_workspace",
           "mc_logdet", "mc_profile_enable", "mc_profile_read",
           "mc_logdet_batched_workspace", "mc_logdet_batched", "mc_tune_get",
           "mc_tune_set", "mc_autotune_workspace", "mc_autotune_batched",
           "mc_last_hip_error", "mc_logdet_factor_workspace",
           "mc_logdet_factor", "mc_logdet_backward_workspace",
           "mc_logdet_backward", "mc_lookahead_enable", "mc_default_panel",
           "mc_split_panel_enable", "mc_logdet_pivots",
           "mc_logdet_backward_recompute_workspace",
           "mc_logdet_backward_recompute", "mc_logdet_rule",
           "mc_logdet_noalloc", "mc_logdet_batched_factor_workspace",
           "mc_logdet_batched_factor", "mc_logdet_batched_backward_workspace",
           "mc_logdet_batched_backward", "mc_gmm_loglik_workspace",
           "mc_gmm_loglik", "mc_batched_spare_xcd0")
INFO_BADARG = -3
TUNE_BUCKETS = (64, 128, 256, 512, 1024, None)  # upper size of each bucket


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
    L.mc_last_hip_error.restype = ctypes.c_char_p
    L.mc_logdet_workspace.argtypes = [i64, ctypes.c_int, ctypes.c_int, i64]
    L.mc_logdet_workspace.restype = sz
    L.mc_logdet.argtypes = [vp, i64, i64, ctypes.c_int, ctypes.c_int, i64, vp,
                            vp, sz, vp]
    L.mc_logdet.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    L.mc_default_panel.argtypes = [ctypes.c_int64, ctypes.c_int]
    L.mc_default_panel.restype = ctypes.c_int64
    L.mc_lookahead_enable.argtypes = [ctypes.c_int]
    L.mc_lookahead_enable.restype = ctypes.c_int
    L.mc_split_panel_enable.argtypes = [ctypes.c_int]
    L.mc_split_panel_enable.restype = ctypes.c_int
    L.mc_profile_enable.argtypes = [ctypes.c_int]
    L.mc_profile_enable.restype = ctypes.c_int
    L.mc_profile_read.argtypes = [ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64), dp, dp]
    L.mc_profile_read.restype = ctypes.c_int
    ci = ctypes.c_int
    L.mc_logdet_batched_workspace.argtypes = [i64, i64, ci, ci, i64]
    L.mc_logdet_batched_workspace.restype = sz
    L.mc_logdet_batched.argtypes = [vp, vp, vp, i64, i64, ci, ci, i64, vp, vp,
                                    sz, vp]
    L.mc_logdet_batched.restype = ci
    i64p = ctypes.POINTER(ctypes.c_int64)
    cip = ctypes.POINTER(ctypes.c_int)
    L.mc_tune_get.argtypes = [ci, ci, i64p, cip]
    L.mc_tune_get.restype = ci
    L.mc_tune_set.argtypes = [ci, ci, i64p, cip]
    L.mc_tune_set.restype = ci
    L.mc_autotune_workspace.argtypes = [ci, i64]
    L.mc_autotune_workspace.restype = sz
    L.mc_autotune_batched.argtypes = [ci, ci, i64, vp, sz, vp]
    L.mc_autotune_batched.restype = ci
    L.mc_logdet_factor_workspace.argtypes = [i64, ci, ci, i64]
    L.mc_logdet_factor_workspace.restype = sz
    L.mc_logdet_factor.argtypes = [vp, i64, i64, ci, ci, i64, vp, vp, vp, sz,
                                   vp]
    L.mc_logdet_factor.restype = ci
    L.mc_logdet_backward_workspace.argtypes = [i64, ci]
    L.mc_logdet_backward_workspace.restype = sz
    L.mc_logdet_backward.argtypes = [vp, i64, i64, vp, ci, vp, vp, vp, i64, vp,
                                     sz, vp]
    L.mc_logdet_backward.restype = ci
    L.mc_logdet_pivots.argtypes = [vp, i64, i64, ci, ci, i64, vp, vp, vp, sz, vp]
    L.mc_logdet_pivots.restype = ci
    L.mc_logdet_backward_recompute_workspace.argtypes = [i64, ci, ci, i64]
    L.mc_logdet_backward_recompute_workspace.restype = sz
    L.mc_logdet_backward_recompute.argtypes = [vp, i64, i64, ci, ci, i64, vp, vp,
                                               i64, vp, vp, sz, vp]
    L.mc_logdet_backward_recompute.restype = ci
    L.mc_logdet_rule.argtypes = [vp, i64, i64, ci, vp, vp, vp, sz, vp]
    L.mc_logdet_rule.restype = ci
    L.mc_logdet_noalloc.argtypes = [vp, i64, i64, ci, ci, i64, vp, vp]
    L.mc_logdet_noalloc.restype = ci
    L.mc_logdet_batched_factor_workspace.argtypes = [i64, i64, ci, ci, i64]
    L.mc_logdet_batched_factor_workspace.restype = sz
    L.mc_logdet_batched_factor.argtypes = [vp, vp, vp, vp, i64, i64, ci, ci, i64,
                                           vp, vp, sz, vp]
    L.mc_logdet_batched_factor.restype = ci
    L.mc_logdet_batched_backward_workspace.argtypes = [i64, i64, ci]
    L.mc_logdet_batched_backward_workspace.restype = sz
    L.mc_logdet_batched_backward.argtypes = [vp, vp, vp, vp, i64, i64, ci, vp, vp,
                                             vp, vp, vp, sz, vp]
    L.mc_logdet_batched_backward.restype = ci
    L.mc_gmm_loglik_workspace.argtypes = [i64, i64, i64, ci]
    L.mc_gmm_loglik_workspace.restype = sz
    L.mc_gmm_loglik.argtypes = [vp, i64, i64, i64, vp, i64, i64, vp, vp, vp, vp,
                                vp, ci, vp, vp, vp, sz, vp]
    L.mc_gmm_loglik.restype = ci
    L.mc_batched_spare_xcd0.argtypes = [ci]
    L.mc_batched_spare_xcd0.restype = ci
    _lib = L
    return L


def _check(status: int, what: str) -> None:
    if status != 0:
        msg = lib().mc_status_string(status).decode()
        if status == -101:
            msg += ": " + lib().mc_last_hip_error().decode()
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


def slogdet_pivots(a: torch.Tensor, b: int = 0, update="native"):
    """(Result, piv_col): piv_col[s] is the original column of the pivot
    taken at step s (an int32 device tensor of n entries).  Synchronises."""
    n = a.shape[0]
    lda = _square_rows(a)
    result = new_result(a.device)
    work = new_workspace(n, a.device, a.dtype, update, b)
    piv = torch.full((max(n, 1),), -1, dtype=torch.int32, device=a.device)
    st = lib().mc_logdet_pivots(a.data_ptr(), n, lda, _dtype_code(a),
                                _update_code(update), b, piv.data_ptr(),
                                result.data_ptr(), work.data_ptr(), work.numel(),
                                _stream_ptr(None, a.device))
    _check(st, "mc_logdet_pivots")
    return read_result(result)[0], piv[:n]


def slogdet_rule(a: torch.Tensor, rule="maxabs"):
    """(Result, piv_col) of the plain FP64 condensation under a pivot-column
    rule: "maxabs" (the paper's, Section 2.2), "first_nonzero" or
    "closest_to_one" (the earlier rules of Section 1).  Synchronises."""
    n = a.shape[0]
    lda = _square_rows(a)
    if a.dtype != torch.float64:
        raise TypeError("the pivot-rule path takes FP64 matrices")
    code = _RULES[rule] if isinstance(rule, str) else int(rule)
    result = new_result(a.device)
    work = new_workspace(n, a.device, torch.float64, "native", 0)
    piv = torch.full((max(n, 1),), -1, dtype=torch.int32, device=a.device)
    st = lib().mc_logdet_rule(a.data_ptr(), n, lda, code, piv.data_ptr(),
                              result.data_ptr(), work.data_ptr(), work.numel(),
                              _stream_ptr(None, a.device))
    _check(st, "mc_logdet_rule")
    return read_result(result)[0], piv[:n]


class Profile(NamedTuple):
    elapsed_ms: float
    launches: int
    alg_bytes: float
    alg_flops: float


def default_panel(n: int, dtype=torch.float64) -> int:
    """Panel width the blocked path takes for b < 0 on an n x n matrix."""
    return int(lib().mc_default_panel(n, _dtype_of(dtype)))


def lookahead_enable(on: bool = True) -> bool:
    """Lookahead on the blocked path (the default): beside each
    column-split panel, the previous panel's trailing update beyond that
    panel's rows runs on a second stream, on the XCDs the panel leaves free.
    Off keeps every kernel on the caller's stream.  Returns the previous
    setting."""
    return bool(lib().mc_lookahead_enable(1 if on else 0))


def split_panel_enable(on: bool = True) -> bool:
    """Blocked panels up to 8192 wide on the column-split kernel (the
    default) or on the row-per-block kernels; returns the previous
    setting."""
    return bool(lib().mc_split_panel_enable(1 if on else 0))


def profile_enable(on: bool = True) -> None:
    """Start (resetting) or stop event timing of the dominant kernel."""
    _check(lib().mc_profile_enable(1 if on else 0), "mc_profile_enable")


def profile_read(kind: str = "update") -> Profile:
    """Summed event timing and algorithmic work of one kind of kernel since
    profile_enable: "update" (trailing update / plain step loop) or
    "panel" (the blocked path's panel-chain kernel)."""
    k = {"update": 0, "panel": 1}[kind]
    ms, la = ctypes.c_double(), ctypes.c_int64()
    by, fl = ctypes.c_double(), ctypes.c_double()
    _check(lib().mc_profile_read(k, ctypes.byref(ms), ctypes.byref(la),
                                 ctypes.byref(by), ctypes.byref(fl)),
           "mc_profile_read")
    return Profile(ms.value, la.value, by.value, fl.value)


# ------------------------------------------------------------------ batched

def _dtype_of(t) -> int:
    return DTYPE_F64 if t == torch.float64 else DTYPE_F32


class BatchedPlan:
    """Device-side description of a batch (pointer, size and stride arrays,
    workspaces, results).  The matrices must stay alive and in place while
    the plan is used.  ``run()`` enqueues the calls on the current stream;
    ``capture()`` records them into a hipGraph (through torch.cuda.CUDAGraph)
    that ``replay()`` launches.

    Members of at least ``blocked_min_n`` rows go through the single-matrix
    blocked path (mc_logdet, one after another, sharing one workspace), the
    rest through one persistent mc_logdet_batched launch: the batched kernel
    condenses each matrix in one workgroup, which for the largest members
    takes longer than the whole-GPU blocked path does for all of them.
    When there are both, the batched launch runs on a second stream beside
    the blocked calls, on the XCDs their column-split panels leave free
    (mc_batched_spare_xcd0); ``concurrent=False`` runs them one after the
    other.  ``blocked_min_n=None`` keeps every member in the batched
    launch."""

    # 64 Wishart members n ~ U{256..2048}, FP64, graph replay: 1280 -> 88.7 ms,
    # 1408 -> 81.3, 1472 -> 67.9, 1536 -> 68.0, 1600 -> 68.2, 1728 -> 88.5;
    # every member batched: 148 (measured with an older batched kernel)
    BLOCKED_MIN_N = 1536

    def __init__(self, mats, b: int = -1, update="native",
                 blocked_min_n: Optional[int] = BLOCKED_MIN_N,
                 concurrent: bool = True):
        if not mats:
            raise ValueError("empty batch")
        dev = mats[0].device
        dt = mats[0].dtype
        for m in mats:
            if m.dtype != dt or m.device != dev:
                raise ValueError("all matrices need one dtype and device")
            _square_rows(m)
        self.mats = list(mats)
        self.device = dev
        self.dtype = dt
        self.b = b
        self.update = _update_code(update)
        self.batch = len(mats)
        ns = [m.shape[0] for m in mats]
        self.large = [i for i, n in enumerate(ns)
                      if blocked_min_n is not None and n >= blocked_min_n]
        big = set(self.large)
        self.small = [i for i in range(self.batch) if i not in big]
        self.result = new_result(dev, self.batch)  # the large members' slots
        self.blocked_work = None
        if self.large:
            n_big = max(ns[i] for i in self.large)
            nb = lib().mc_logdet_workspace(n_big, _dtype_of(dt), self.update, -1)
            if nb == 0:
                raise MCError("unsupported combination for the blocked path")
            self.blocked_work = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.n_max = max([ns[i] for i in self.small], default=0)
        if self.small:
            sm = [mats[i] for i in self.small]
            self.ptrs = torch.tensor([m.data_ptr() for m in sm], dtype=torch.int64,
                                     device=dev)
            self.ns = torch.tensor([m.shape[0] for m in sm], dtype=torch.int64,
                                   device=dev)
            self.ldas = torch.tensor([_square_rows(m) for m in sm], dtype=torch.int64,
                                     device=dev)
            nb = lib().mc_logdet_batched_workspace(len(sm), self.n_max,
                                                   _dtype_of(dt), self.update, b)
            if nb == 0:
                raise MCError("unsupported combination for the batched path")
            self.work = torch.empty(nb, dtype=torch.uint8, device=dev)
            self.small_result = new_result(dev, len(sm))
        self.graph = None
        self.concurrent = concurrent and bool(self.large) and bool(self.small)
        # default priority, as every stream here
        self.side = torch.cuda.Stream(dev) if self.concurrent else None

    def _batched_call(self, sp: int) -> None:
        st = lib().mc_logdet_batched(
            self.ptrs.data_ptr(), self.ns.data_ptr(), self.ldas.data_ptr(),
            len(self.small), self.n_max, _dtype_of(self.dtype), self.update,
            self.b, self.small_result.data_ptr(), self.work.data_ptr(),
            self.work.numel(), sp)
        _check(st, "mc_logdet_batched")

    def run(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        main = stream if stream is not None else torch.cuda.current_stream(self.device)
        sp = main.cuda_stream
        if self.concurrent:
            # the small members on the side stream, off XCD 0, beside the
            # large members' blocked calls on this one
            self.side.wait_stream(main)
            old = lib().mc_batched_spare_xcd0(1)
            try:
                self._batched_call(self.side.cuda_stream)
            finally:
                lib().mc_batched_spare_xcd0(old)
        for i in self.large:
            m = self.mats[i]
            st = lib().mc_logdet(m.data_ptr(), m.shape[0], _square_rows(m),
                                 _dtype_of(self.dtype), self.update, -1,
                                 self.result[i:i + 1].data_ptr(),
                                 self.blocked_work.data_ptr(),
                                 self.blocked_work.numel(), sp)
            _check(st, "mc_logdet")
        if self.concurrent:
            main.wait_stream(self.side)
        elif self.small:
            self._batched_call(sp)

    def capture(self) -> None:
        self.run()  # warm-up outside the capture (kernel attributes)
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g

    def replay(self) -> None:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def results(self) -> list:
        out = read_result(self.result)
        if self.small:
            for i, r in zip(self.small, read_result(self.small_result)):
                out[i] = r
        return out


def _ptr_array(tensors, device) -> torch.Tensor:
    return torch.tensor([t.data_ptr() for t in tensors], dtype=torch.int64,
                        device=device)


def factor_batched(mats, b: int = -1, update="native"):
    """Factor copies of the matrices in one persistent launch
    (mc_logdet_batched_factor): returns (lus, perms, result) with
    mats[k][:, perms[k]] = L U (L\\U in lus[k]) and result the device buffer
    of the batch's mc_result structs (not yet synchronised)."""
    if not mats:
        raise ValueError("empty batch")
    dev, dt = mats[0].device, mats[0].dtype
    lus = [m.detach().contiguous().clone() for m in mats]
    for m in lus:
        _square_rows(m)
        if m.dtype != dt or m.device != dev:
            raise ValueError("all matrices need one dtype and device")
    ns = [m.shape[0] for m in lus]
    perms = [torch.empty(max(n, 1), dtype=torch.int32, device=dev) for n in ns]
    n_max = max(ns)
    nb = lib().mc_logdet_batched_factor_workspace(len(lus), n_max, _dtype_of(dt),
                                                 _update_code(update), b)
    if nb == 0:
        raise MCError("unsupported combination for the batched factor call")
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    res = new_result(dev, len(lus))
    ptrs = _ptr_array(lus, dev)
    nsd = torch.tensor(ns, dtype=torch.int64, device=dev)
    ldas = torch.tensor([max(n, 1) for n in ns], dtype=torch.int64, device=dev)
    pp = _ptr_array(perms, dev)
    st = lib().mc_logdet_batched_factor(
        ptrs.data_ptr(), nsd.data_ptr(), ldas.data_ptr(), pp.data_ptr(), len(lus),
        n_max, _dtype_of(dt), _update_code(update), b, res.data_ptr(),
        work.data_ptr(), work.numel(), _stream_ptr(None, dev))
    _check(st, "mc_logdet_batched_factor")
    return lus, [p[:n] for p, n in zip(perms, ns)], res


def backward_batched(lus, perms, grad_out: Optional[torch.Tensor] = None,
                     fwd: Optional[torch.Tensor] = None) -> list:
    """g_k * A_k^{-T} for every member from stored factors, in one persistent
    launch (mc_logdet_batched_backward).  grad_out: device float64 tensor of
    one entry per member (None: 1); fwd: the factor calls' device results
    (members whose info != 0 get an all-NaN gradient)."""
    if not lus:
        return []
    dev, dt = lus[0].device, lus[0].dtype
    ns = [m.shape[0] for m in lus]
    n_max = max(ns)
    grads = [torch.empty_like(m) for m in lus]
    nb = lib().mc_logdet_batched_backward_workspace(len(lus), n_max, _dtype_of(dt))
    if nb == 0:
        raise MCError("unsupported combination for the batched backward call")
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    lp = _ptr_array(lus, dev)
    gp = _ptr_array(grads, dev)
    pp = _ptr_array(perms, dev)
    nsd = torch.tensor(ns, dtype=torch.int64, device=dev)
    lds = torch.tensor([_square_rows(m) for m in lus], dtype=torch.int64, device=dev)
    ldg = torch.tensor([_square_rows(g) for g in grads], dtype=torch.int64, device=dev)
    g_ptr = None
    if grad_out is not None:
        grad_out = grad_out.detach().to(dev, torch.float64).contiguous()
        g_ptr = grad_out.data_ptr()
    st = lib().mc_logdet_batched_backward(
        lp.data_ptr(), nsd.data_ptr(), lds.data_ptr(), pp.data_ptr(), len(lus),
        n_max, _dtype_of(dt), g_ptr, fwd.data_ptr() if fwd is not None else None,
        gp.data_ptr(), ldg.data_ptr(), work.data_ptr(), work.numel(),
        _stream_ptr(None, dev))
    _check(st, "mc_logdet_batched_backward")
    return grads


def logdet_batched(mats, b: int = -1, update="native") -> list:
    """(sign, log|det|, info) of every matrix of a batch (synchronises)."""
    plan = BatchedPlan(mats, b=b, update=update)
    plan.run()
    return plan.results()


def tune_get(dtype=torch.float64, update="native"):
    b = (ctypes.c_int64 * 6)()
    t = (ctypes.c_int * 6)()
    _check(lib().mc_tune_get(_dtype_of(dtype), _update_code(update), b, t),
           "mc_tune_get")
    return list(b), list(t)


def tune_set(b_list, tile_list, dtype=torch.float64, update="native"):
    b = (ctypes.c_int64 * 6)(*b_list)
    t = (ctypes.c_int * 6)(*tile_list)
    _check(lib().mc_tune_set(_dtype_of(dtype), _update_code(update), b, t),
           "mc_tune_set")


def autotune_batched(dtype=torch.float64, update="native", n_max: int = 1024,
                     device=None):
    """Run the library's autotuner for the batched path; returns the table."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    nb = lib().mc_autotune_workspace(_dtype_of(dtype), n_max)
    if nb == 0:
        raise MCError("unsupported autotune request")
    work = torch.empty(nb, dtype=torch.uint8, device=device)
    _check(lib().mc_autotune_batched(_dtype_of(dtype), _update_code(update),
                                     n_max, work.data_ptr(), work.numel(),
                                     _stream_ptr(None, device)),
           "mc_autotune_batched")
    del work
    return tune_get(dtype, update)


def _tune_key(dtype, update, n_max: int, device) -> str:
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "")
    return (f"{props.name}|{arch}|cu{props.multi_processor_count}|"
            f"v{lib().mc_version()}|{'f64' if _dtype_of(dtype) == DTYPE_F64 else 'f32'}|"
            f"u{_update_code(update)}|n{n_max}")


def default_tune_cache() -> str:
    base = os.environ.get("MC_TUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1811_08057_amd",
                        "tune.json")


def load_tune_entry(path: str, key: str):
    """(b list, tile list) stored under `key` in the cache file, or None when
    the file is missing, unreadable or holds no valid entry for the key."""
    import json
    try:
        with open(path) as f:
            data = json.load(f)
        e = data[key]
        b, t = [int(x) for x in e["b"]], [int(x) for x in e["tile"]]
        if len(b) != len(TUNE_BUCKETS) or len(t) != len(TUNE_BUCKETS):
            return None
        return b, t
    except (OSError, ValueError, KeyError, TypeError):
        return None


def store_tune_entry(path: str, key: str, b, tile) -> bool:
    """Add or replace one entry of the cache file (written atomically)."""
    import json
    try:
        data = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if not isinstance(data, dict):
                data = {}
    except (OSError, ValueError):
        data = {}
    data[key] = {"b": list(b), "tile": list(tile)}
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, path)
        return True
    except OSError:
        return False


def autotune_cached(dtype=torch.float64, update="native", n_max: int = 1024,
                    device=None, cache: Optional[str] = None):
    """The batched path's tuning table for this device, set in the library
    and returned with where it came from ("cache", "tuned" or "default"):
    the cache file's entry for this device, library version, dtype, update
    and n_max when there is one; else mc_autotune_batched now, stored in
    the cache; the library's defaults if tuning fails."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    path = cache or default_tune_cache()
    key = _tune_key(dtype, update, n_max, device)
    hit = load_tune_entry(path, key)
    if hit is not None:
        try:
            tune_set(hit[0], hit[1], dtype, update)
            return hit[0], hit[1], "cache"
        except MCError:
            pass  # an entry the library rejects: tune afresh
    try:
        b, t = autotune_batched(dtype, update, n_max, device)
    except (MCError, RuntimeError):
        b, t = tune_get(dtype, update)
        return b, t, "default"
    store_tune_entry(path, key, b, t)
    return b, t, "tuned"


# ------------------------------------------------------- factor / backward

def factor(a: torch.Tensor, b: int = -1, update="native"):
    """Factor a copy of `a` in place: returns (lu, perm, result) where
    a[:, perm] = L U (L\\U stored in lu) and result is the device mc_result
    buffer (not yet synchronised)."""
    n = a.shape[0]
    lu = a.detach().contiguous().clone()
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=a.device)
    res = new_result(a.device)
    nb = lib().mc_logdet_factor_workspace(n, _dtype_code(a), _update_code(update),
                                          b)
    if nb == 0:
        raise MCError("unsupported combination for the factor call")
    work = torch.empty(nb, dtype=torch.uint8, device=a.device)
    st = lib().mc_logdet_factor(lu.data_ptr(), n, max(n, 1), _dtype_code(a),
                                _update_code(update), b, perm.data_ptr(),
                                res.data_ptr(), work.data_ptr(), work.numel(),
                                _stream_ptr(None, a.device))
    _check(st, "mc_logdet_factor")
    return lu, perm[:n], res


def backward(lu: torch.Tensor, perm: torch.Tensor,
             grad_out: Optional[torch.Tensor] = None,
             fwd: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g * A^{-T} from factor()'s output; grad_out: device float64 scalar;
    fwd: the factor call's device result (NaN gradient when its info != 0)."""
    n = lu.shape[0]
    grad = torch.empty_like(lu)
    nb = lib().mc_logdet_backward_workspace(n, _dtype_code(lu))
    work = torch.empty(max(nb, 1), dtype=torch.uint8, device=lu.device)
    g_ptr = None
    if grad_out is not None:
        grad_out = grad_out.detach().to(lu.device, torch.float64).contiguous()
        g_ptr = grad_out.data_ptr()
    st = lib().mc_logdet_backward(lu.data_ptr(), n, max(n, 1), perm.data_ptr(),
                                  _dtype_code(lu), g_ptr,
                                  fwd.data_ptr() if fwd is not None else None,
                                  grad.data_ptr(), max(n, 1), work.data_ptr(),
                                  work.numel(), _stream_ptr(None, lu.device))
    _check(st, "mc_logdet_backward")
    return grad


def backward_recompute(a: torch.Tensor, grad_out: Optional[torch.Tensor] = None,
                       b: int = -1, update="native",
                       out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g * A^{-T} with the factors recomputed from A inside the library's
    workspace (mc_logdet_backward_recompute); out: optional device result."""
    n = a.shape[0]
    lda = _square_rows(a)
    grad = torch.empty((n, n), dtype=a.dtype, device=a.device)
    nb = lib().mc_logdet_backward_recompute_workspace(n, _dtype_code(a),
                                                      _update_code(update), b)
    if nb == 0 and n > 0:
        raise MCError("unsupported combination for the recompute call")
    work = torch.empty(max(nb, 1), dtype=torch.uint8, device=a.device)
    g_ptr = None
    if grad_out is not None:
        grad_out = grad_out.detach().to(a.device, torch.float64).contiguous()
        g_ptr = grad_out.data_ptr()
    st = lib().mc_logdet_backward_recompute(
        a.data_ptr(), n, lda, _dtype_code(a), _update_code(update), b, g_ptr,
        grad.data_ptr(), max(n, 1), out.data_ptr() if out is not None else None,
        work.data_ptr(), work.numel(), _stream_ptr(None, a.device))
    _check(st, "mc_logdet_backward_recompute")
    return grad


class MCLogDet(torch.autograd.Function):
    """(sign, log|det A|) with d log|det A| / dA = A^{-T}.

    forward keeps the factors (L\\U and perm) when they fit `mem_budget`
    bytes (None = always); otherwise backward recomputes them from A in the
    library (mc_logdet_backward_recompute).  A failed factorisation
    (singular, non-finite) gives logabsdet -inf or NaN in forward and an
    all-NaN gradient in backward, decided on the device from the forward's
    info (no host synchronisation)."""

    @staticmethod
    def forward(ctx, a, b=-1, update="native", mem_budget=None):
        lu, perm, res = factor(a, b=b, update=update)
        keep = mem_budget is None or lu.numel() * lu.element_size() <= mem_budget
        if keep:
            ctx.save_for_backward(lu, perm, res)
        else:
            del lu, perm
            ctx.save_for_backward(a.detach())
        ctx.keep = keep
        ctx.b, ctx.update = b, update
        sign = res[0, 1].clone()
        logabs = res[0, 0].clone()
        ctx.mark_non_differentiable(sign)
        return sign, logabs

    @staticmethod
    def backward(ctx, gsign, glogabs):
        if ctx.keep:
            lu, perm, res = ctx.saved_tensors
            g = backward(lu, perm, glogabs, fwd=res)
        else:
            (a,) = ctx.saved_tensors
            g = backward_recompute(a, glogabs, b=ctx.b, update=ctx.update)
        return g, None, None, None


def slogdet_autograd(a: torch.Tensor, b: int = -1, update="native",
                     mem_budget: Optional[int] = None):
    """Differentiable (sign, log|det A|) as device tensors (no host sync)."""
    return MCLogDet.apply(a, b, update, mem_budget)


# ------------------------------------------------------ batched autograd

class MCLogDetBatched(torch.autograd.Function):
    """(signs, log|det A_k|) of a batch, with d log|det A_k| / dA_k =
    A_k^{-T}.  Forward keeps every member's factors: members of at least
    ``BatchedPlan.BLOCKED_MIN_N`` rows through the single-matrix factor call
    (the whole-GPU blocked path), the rest through one batched factor
    launch.  Backward is one batched backward launch over all members
    (failed members get NaN gradients, decided on the device)."""

    @staticmethod
    def forward(ctx, b, update, *mats):
        mats = [m.detach() for m in mats]
        dev = mats[0].device
        big = [k for k, m in enumerate(mats) if m.shape[0] >= BatchedPlan.BLOCKED_MIN_N]
        small = [k for k in range(len(mats)) if k not in set(big)]
        lus = [None] * len(mats)
        perms = [None] * len(mats)
        res = [None] * len(mats)
        main = torch.cuda.current_stream(dev)
        side = None
        if small and big:
            # the small members' batched factor launch on a second stream,
            # off XCD 0, beside the large members' blocked factor calls
            side = torch.cuda.Stream(dev)
            side.wait_stream(main)
            with torch.cuda.stream(side):
                old = lib().mc_batched_spare_xcd0(1)
                try:
                    sl, sp, sr = factor_batched([mats[k] for k in small], b=b,
                                                update=update)
                finally:
                    lib().mc_batched_spare_xcd0(old)
        elif small:
            sl, sp, sr = factor_batched([mats[k] for k in small], b=b, update=update)
        for k in big:
            lus[k], perms[k], res[k] = factor(mats[k], b=b, update=update)
        if side is not None:
            main.wait_stream(side)
            for t in [*sl, *sp, sr]:
                t.record_stream(main)  # made on the side stream, used here
        if small:
            for i, k in enumerate(small):
                lus[k], perms[k], res[k] = sl[i], sp[i], sr[i:i + 1]
        fwd = torch.cat(res).to(dev)
        ctx.save_for_backward(fwd, *lus, *perms)
        ctx.count = len(mats)
        signs = fwd[:, 1].clone()
        logabs = fwd[:, 0].clone()
        ctx.mark_non_differentiable(signs)
        return signs, logabs

    @staticmethod
    def backward(ctx, gsigns, glogabs):
        saved = ctx.saved_tensors
        fwd, c = saved[0], ctx.count
        lus, perms = list(saved[1:1 + c]), list(saved[1 + c:1 + 2 * c])
        if glogabs is None:
            glogabs = torch.zeros(c, dtype=torch.float64, device=fwd.device)
        grads = backward_batched(lus, perms, grad_out=glogabs, fwd=fwd)
        return (None, None, *grads)


def slogdet_batched_autograd(mats, b: int = -1, update="native"):
    """Differentiable (signs, log|det|) of a list of device matrices, as two
    device tensors of len(mats) entries (no host synchronisation)."""
    return MCLogDetBatched.apply(b, update, *mats)


# ------------------------------------------------- mixture log-likelihood

class GmmFactors(NamedTuple):
    """Each component's kept factors (as the factor calls leave them)."""
    lus: list
    perms: list
    fwd: torch.Tensor  # (k, 3) device mc_result structs


def gmm_factor(covs, update="native") -> GmmFactors:
    """Factor the mixture's covariances: one batched factor launch, or the
    blocked factor call per component from BatchedPlan.BLOCKED_MIN_N rows
    (the whole-GPU path for large dimensions)."""
    d = covs[0].shape[0]
    if d >= BatchedPlan.BLOCKED_MIN_N:
        outs = [factor(c, update=update) for c in covs]
        return GmmFactors([o[0] for o in outs], [o[1] for o in outs],
                          torch.cat([o[2] for o in outs]))
    lus, perms, res = factor_batched(list(covs), update=update)
    return GmmFactors(lus, perms, res)


def gmm_loglik(x: torch.Tensor, log_weights: torch.Tensor, means: torch.Tensor,
               fac: GmmFactors, with_total: bool = True):
    """Per-point log-likelihood (m doubles) and its sum (or None) of a
    Gaussian mixture from its factored covariances (mc_gmm_loglik).  x: m x d,
    means: k x d (the factors' dtype); log_weights: k (log pi_k)."""
    m, d = x.shape
    k = means.shape[0]
    dev = x.device
    if x.stride(1) != 1 or means.stride(1) != 1:
        raise ValueError("rows must be contiguous")
    lw = log_weights.detach().to(dev, torch.float64).contiguous()
    out = torch.empty(max(m, 1), dtype=torch.float64, device=dev)
    total = torch.empty(1, dtype=torch.float64, device=dev) if with_total else None
    nb = lib().mc_gmm_loglik_workspace(m, d, k, _dtype_code(x))
    if nb == 0:
        raise MCError("unsupported mixture size")
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    lp = _ptr_array(fac.lus, dev)
    pp = _ptr_array(fac.perms, dev)
    lds = torch.tensor([_square_rows(u) for u in fac.lus], dtype=torch.int64, device=dev)
    st = lib().mc_gmm_loglik(
        x.data_ptr(), m, d, max(x.stride(0), d), means.data_ptr(),
        max(means.stride(0), d), k, lw.data_ptr(), lp.data_ptr(), lds.data_ptr(),
        pp.data_ptr(), fac.fwd.data_ptr(), _dtype_code(x), out.data_ptr(),
        total.data_ptr() if total is not None else None, work.data_ptr(),
        work.numel(), _stream_ptr(None, dev))
    _check(st, "mc_gmm_loglik")
    return out[:m], total
