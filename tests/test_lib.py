"""The C-ABI library loads and exports every entry point include/dfm.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfm.h")
LIB = os.path.join(ROOT, "paper_1608_04607_amd", "libdfm.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for n in ("dfm_mesh_build", "dfm_assemble", "dfm_solve", "dfm_apply", "dfm_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfm.so not built")
def test_binding_declares_every_header_symbol():
    from paper_1608_04607_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_symbols()
    _lib.load()
