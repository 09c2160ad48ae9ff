"""The C-ABI library builds, loads and exports every declared entry point
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ucov.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char \*)\s*(ucov_\w+)\s*\(", text, re.M)))


def test_header_declares_the_binding_exports():
    from paper_1808_02414_amd import _binding
    assert declared_functions() == sorted(_binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1808_02414_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libucov.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib2 = _binding.load()
    assert lib2.ucov_strerror(-3).decode().startswith("regularised")
