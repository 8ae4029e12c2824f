"""The C-ABI library loads and exports every entry point include/sa.h declares
(no GPU needed; no compute calls)."""

import ctypes
import os
import re

import pytest

from paper_1610_03007_amd import _native, build_ext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(sa_[a-z0-9_]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("sa_ctx_create", "sa_ctx_destroy", "sa_build", "sa_radix_sort_pairs",
                 "sa_strerror", "sa_workspace_bytes"):
        assert must in names
    assert sorted(_native.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(build_ext.LIB if os.path.exists(build_ext.LIB) else _native.lib()._name)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_entry_points():
    lib = _native.lib()
    assert lib.sa_strerror(0).decode() == "ok"
    assert "2^32" in lib.sa_strerror(3).decode()
    n = 1 << 20
    ws = lib.sa_workspace_bytes(n, 1)
    assert 36 * n <= ws <= 40 * n
    assert lib.sa_workspace_bytes(n, 0) == ws
    # A batch adds 8 bytes per position for its survivors and a table row per text.
    wb = lib.sa_workspace_bytes(n, 4096)
    assert ws + 8 * n + 4096 * 597 <= wb <= ws + 8 * n + 4096 * 700
    assert ws + 8 * n <= lib.sa_workspace_bytes(n, 2) <= ws + 8 * n + 2 * 700 + 4096


def test_null_context_is_rejected():
    lib = _native.lib()
    assert lib.sa_build(None, None, 10, 4, None, None) == _native.SA_EINVAL
    assert lib.sa_radix_sort_pairs(None, None, None, 10, 8, None) == _native.SA_EINVAL
    assert lib.sa_ctx_create(None, 0, None) == _native.SA_EINVAL
    assert lib.sa_ctx_destroy(None) == _native.SA_OK
