"""The C-ABI library loads on the CPU-only host and exports every symbol the
header declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2306_09189_amd import hecnn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "hecnn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b((?:hec|ckks|he)_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_matches_binding_list():
    assert declared() == set(hecnn.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(hecnn.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(hecnn.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name
    hecnn.lib()  # signatures attach


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(hecnn, "_lib", None)
    monkeypatch.setattr(hecnn, "LIB_PATH", "/nonexistent/libhecnn.so")
    with pytest.raises(RuntimeError):
        hecnn.lib()
