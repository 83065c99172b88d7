"""The C ABI on the CPU: the built library loads and exports every function
that include/hnsearch.h declares, and the binding's signature table matches
the header.  No compute call is made here (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hnsearch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hn_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hn_build_index", "hn_search_top1", "hn_bruteforce_top1", "hn_free_index",
                 "hn_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2606_27280_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhnsearch.so is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_the_header():
    from paper_2606_27280_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2606_27280_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()


def test_error_message_api_without_gpu():
    from paper_2606_27280_amd import _lib
    L = _lib.lib()
    # argument validation happens before any device work
    h = ctypes.c_void_p()
    rc = L.hn_build_index(None, 10, 128, 8, 0.1, 0, None, ctypes.byref(h))
    assert rc == _lib.HN_ERR_INVALID_ARG
    assert b"null" in L.hn_last_error()
    rc = L.hn_build_index(ctypes.c_void_p(16), 10, 64, 8, 0.1, 0, None, ctypes.byref(h))
    assert rc == _lib.HN_ERR_INVALID_ARG and b"128" in L.hn_last_error()
    rc = L.hn_build_index(ctypes.c_void_p(16), 10, 128, 0, 0.1, 0, None, ctypes.byref(h))
    assert rc == _lib.HN_ERR_INVALID_ARG
    rc = L.hn_build_index(ctypes.c_void_p(16), 10, 128, 8, 1.0, 0, None, ctypes.byref(h))
    assert rc == _lib.HN_ERR_INVALID_ARG
    rc = L.hn_search_top1(None, None, 0, None, None, None, None, None, None)
    assert rc == _lib.HN_ERR_INVALID_ARG
    rc = L.hn_bruteforce_top1(ctypes.c_void_p(16), 10, 100, None, 0, None, None, None)
    assert rc == _lib.HN_ERR_INVALID_ARG


def test_memory_budget_and_noalloc_argument_checks_without_gpu():
    from paper_2606_27280_amd import _lib
    L = _lib.lib()
    assert L.hn_memory_held() == 0
    assert L.hn_set_memory_budget(-1) == _lib.HN_ERR_INVALID_ARG
    assert L.hn_set_memory_budget(0) == _lib.HN_OK
    rc = L.hn_search_top1_noalloc(None, None, 0, None, None, None, None, None)
    assert rc == _lib.HN_ERR_INVALID_ARG and b"null" in L.hn_last_error()
    h = ctypes.c_void_p()
    rc = L.hn_build_index(ctypes.c_void_p(16), 10, 128, 8, 0.1, 1 << 1, None, ctypes.byref(h))
    assert rc == _lib.HN_ERR_INVALID_ARG and b"flags" in L.hn_last_error()
