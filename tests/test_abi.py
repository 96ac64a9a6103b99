"""The C-ABI library loads and exports every symbol its headers declare.

No compute call is made here (no GPU in this environment); only the
host-side argument checks, which return before anything is enqueued.
"""

import ctypes
import glob
import os
import re

import pytest

import paper_1811_08057_amd as mc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mc_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = mc.lib()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), f"{name} not exported"
    assert set(mc.EXPORTS) == declared


def test_version_and_status_strings():
    lib = mc.lib()
    assert lib.mc_version() >= 100
    assert lib.mc_status_string(0) == b"ok"
    assert b"workspace" in lib.mc_status_string(-100)
    assert b"invalid" in lib.mc_status_string(-3)


def test_workspace_queries():
    lib = mc.lib()
    assert lib.mc_logdet_workspace(-1, 0, 0, 0) == 0
    small = lib.mc_logdet_workspace(10, 0, 0, 0)
    big = lib.mc_logdet_workspace(1000, 0, 0, 0)
    assert 0 < small < big
    # the plain path holds the matrix (rows padded to 16 doubles)
    assert big >= 1000 * 1008 * 8


def test_host_argument_checks_return_before_launch():
    lib = mc.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced: checks fail first
    out = ctypes.c_void_p(512)
    # n < 0
    assert lib.mc_logdet(fake, -1, 1, 0, 0, 0, out, fake, 1 << 20, None) == -2
    # A == NULL with n > 0
    assert lib.mc_logdet(None, 4, 4, 0, 0, 0, out, fake, 1 << 20, None) == -1
    # lda < n
    assert lib.mc_logdet(fake, 4, 3, 0, 0, 0, out, fake, 1 << 20, None) == -3
    # bad dtype / update
    assert lib.mc_logdet(fake, 4, 4, 7, 0, 0, out, fake, 1 << 20, None) == -4
    assert lib.mc_logdet(fake, 4, 4, 0, 9, 0, out, fake, 1 << 20, None) == -5
    # out == NULL
    assert lib.mc_logdet(fake, 4, 4, 0, 0, 0, None, fake, 1 << 20, None) == -7
    # workspace missing, misaligned, too small
    assert lib.mc_logdet(fake, 4, 4, 0, 0, 0, out, None, 1 << 20, None) == -8
    assert lib.mc_logdet(fake, 4, 4, 0, 0, 0, out, ctypes.c_void_p(264),
                         1 << 20, None) == -8
    assert lib.mc_logdet(fake, 4, 4, 0, 0, 0, out, fake, 16, None) == -100


def test_binding_rejects_host_tensors():
    import torch
    with pytest.raises(ValueError):
        mc.logdet_async(torch.eye(3, dtype=torch.float64),
                        torch.empty(3, dtype=torch.float64),
                        torch.empty(10, dtype=torch.uint8))


def test_rule_call_argument_checks():
    lib = mc.lib()
    fake = ctypes.c_void_p(256)
    out = ctypes.c_void_p(512)
    piv = ctypes.c_void_p(1024)
    assert lib.mc_logdet_rule(fake, -1, 1, 0, piv, out, fake, 1 << 20, None) == -2
    assert lib.mc_logdet_rule(None, 4, 4, 0, piv, out, fake, 1 << 20, None) == -1
    assert lib.mc_logdet_rule(fake, 4, 3, 0, piv, out, fake, 1 << 20, None) == -3
    for bad_rule in (-1, 3):
        assert lib.mc_logdet_rule(fake, 4, 4, bad_rule, piv, out, fake, 1 << 20,
                                  None) == -4
    assert lib.mc_logdet_rule(fake, 4, 4, 2, piv, None, fake, 1 << 20, None) == -6
    assert lib.mc_logdet_rule(fake, 4, 4, 1, None, out, None, 1 << 20, None) == -7
    assert lib.mc_logdet_rule(fake, 4, 4, 1, None, out, fake, 16, None) == -100


def test_tune_cache_round_trip_and_fallbacks(tmp_path):
    """The tuning-table cache (host side only): an entry stored is read back
    and set in the library; a corrupt file or a malformed entry reads as
    missing (the caller then tunes, or keeps the defaults)."""
    path = str(tmp_path / "tune.json")
    b = [16, 32, 32, 64, 64, 128]
    t = [32, 32, 64, 64, 64, 64]
    assert mc.load_tune_entry(path, "k") is None
    assert mc.store_tune_entry(path, "k", b, t)
    assert mc.load_tune_entry(path, "k") == (b, t)
    assert mc.store_tune_entry(path, "other", t, b)
    assert mc.load_tune_entry(path, "k") == (b, t)
    import torch
    old = mc.tune_get(torch.float64)
    try:
        mc.tune_set(b, t, torch.float64)
        assert mc.tune_get(torch.float64) == (b, t)
    finally:
        mc.tune_set(*old, torch.float64)
    with open(path, "w") as f:
        f.write("{not json")
    assert mc.load_tune_entry(path, "k") is None
    with open(path, "w") as f:
        f.write('{"k": {"b": [1, 2], "tile": [32]}}')
    assert mc.load_tune_entry(path, "k") is None
