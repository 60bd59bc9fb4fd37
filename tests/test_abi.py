"""C ABI checks that need no GPU: the library loads, exports what osog.h declares,
and host-side argument checks return their status before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib():
    from paper_2606_21381_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libosog.so not built")
    return _lib, _lib.load()


def test_exports_match_header():
    _lib, L = lib()
    hdr = open(os.path.join(ROOT, "include", "osog.h")).read()
    declared = set(re.findall(r"\b(osog_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings():
    _lib, L = lib()
    assert L.osog_status_string(0) == b"OSOG_OK"
    assert L.osog_status_string(3) == b"OSOG_ERR_WORKSPACE"


def test_null_context_is_rejected_without_gpu():
    _lib, L = lib()
    o = _lib.Optics()
    assert L.osog_render(None, None, 64, 64, None, 0, 0, ctypes.byref(o), None, None, None, None, 0) == 5
    assert L.osog_render_backward(None, None, 64, 64, None, 0, 0, ctypes.byref(o), None, None, None,
                                  None, None, None, 0) == 5
    b = ctypes.c_size_t()
    assert L.osog_workspace_size(None, 64, 64, 10, 0, 0, ctypes.byref(b)) == 5
    assert L.osog_set_tiling(None, 16, 16) == 5
    assert L.osog_context_destroy(None) == 5
    assert b"context" in L.osog_last_error()


def test_philox_argument_checks():
    _lib, L = lib()
    assert L.osog_philox4x32_10(None, None, -1, 0, 0, None) == 1
    assert L.osog_philox4x32_10(None, None, 5, 0, 0, None) == 1
    assert L.osog_philox4x32_10(None, None, 0, 0, 0, None) == 0
