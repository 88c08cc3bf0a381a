"""The C-ABI library loads on the host and exports every function include/sfft.h
declares. No compute call is made here (no GPU in this environment)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfft.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sfft_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("sfft_plan_create", "sfft_apply", "sfft_apply_multi", "sfft_workspace_size",
                 "sfft_plan_info", "sfft_plan_destroy", "sfft_status_string"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2406_17981_amd import _native
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_native.EXPORTS) == _declared()


def test_host_only_calls():
    from paper_2406_17981_amd import _native as N
    assert N.lib.sfft_status_string(N.INVALID_ARG) == b"SFFT_INVALID_ARG"
    assert N.lib.sfft_length_supported(64) == 1
    assert N.lib.sfft_length_supported(7) == 0
    for L in (16, 40, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512, 768, 1024, 2048):
        assert N.lib.sfft_length_supported(L) == 1, L


def test_argument_validation_without_a_device():
    """Validation happens before any HIP call, so it is testable on the host."""
    from paper_2406_17981_amd import _native as N
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(16, 16, 16)
    fake = ctypes.c_void_p(0x1000)
    assert N.lib.sfft_plan_create(None, 3, n, 1, fake, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_create(ctypes.byref(h), 0, n, 1, fake, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_create(ctypes.byref(h), 7, n, 1, fake, 0, 0, None, 1, 0, None) == N.UNSUPPORTED
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n, 2, fake, 0, 0, None, 1, 0, None) == N.UNSUPPORTED
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n, 1, None, 0, 0, None, 1, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n, 1, fake, 5, 0, None, 1, 0, None) == N.INVALID_ARG
    n7 = (ctypes.c_int64 * 3)(16, 7, 16)
    assert N.lib.sfft_plan_create(ctypes.byref(h), 3, n7, 1, fake, 0, 0, None, 1, 0, None) == N.UNSUPPORTED
    assert b"7" in N.lib.sfft_last_error() or b"14" in N.lib.sfft_last_error()
    assert N.lib.sfft_apply(None, fake, fake, 1, None, 0, None) == N.INVALID_ARG
    assert N.lib.sfft_plan_update(None, fake, None) == N.INVALID_ARG
    assert b"null" in N.lib.sfft_last_error()


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle (it is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2406_17981_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", txt, re.M), f
                assert "oracle/" not in txt, f
