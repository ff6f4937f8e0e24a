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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfm.so not built")
def test_every_entry_point_rejects_null_arguments():
    """Every call returns DFM_E_INVALID (-1) with a message for null handles and
    null pointers, before it reaches the HIP runtime (so this runs without a GPU);
    the destroy calls accept NULL."""
    from paper_1608_04607_amd import _lib
    lib = _lib.load()
    ints = (ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_uint32)
    checked = 0
    for name, res, argtypes in _lib._PROTOS:
        if name == "dfm_last_error":
            continue
        args = [0 if t in ints else 0.0 if t in (ctypes.c_double, ctypes.c_float) else None for t in argtypes]
        r = getattr(lib, name)(*args)
        if name.endswith("_destroy"):
            assert r is None
            continue
        assert r == -1, (name, r)
        assert lib.dfm_last_error().startswith(b"null"), name
        checked += 1
    assert checked >= 15
