"""The C-ABI library loads and exports every symbol ``include/ibm.h`` declares.

Runs without a GPU: only argument checks that fail before any HIP call are
exercised here.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ibm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2006_03343_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2006_03343_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    from paper_2006_03343_amd import _lib
    assert set(names) == set(_lib.EXPORTS)


def test_host_argument_checks(lib):
    from paper_2006_03343_amd import _lib
    h = ctypes.c_void_p()
    assert lib.ibm_create(None, None, 0, 0) == _lib.IBM_E_ARG
    assert b"NULL" in lib.ibm_last_error()
    g = _lib.IbmGrid(0, 4, 4, 1.0, 1.0, 1.0)
    assert lib.ibm_create(ctypes.byref(h), ctypes.byref(g), 0, 0) == _lib.IBM_E_ARG
    g = _lib.IbmGrid(4, 4, 4, 1.0, -1.0, 1.0)
    assert lib.ibm_create(ctypes.byref(h), ctypes.byref(g), 0, 0) == _lib.IBM_E_ARG
    g = _lib.IbmGrid(4, 4, 4, 1.0, 1.0, 1.0)
    assert lib.ibm_create(ctypes.byref(h), ctypes.byref(g), 7, 0) == _lib.IBM_E_ARG
    assert lib.ibm_create(ctypes.byref(h), ctypes.byref(g), 1, 1) == _lib.IBM_E_UNSUPPORTED
    g = _lib.IbmGrid(2048, 2048, 1024, 1.0, 1.0, 1.0)
    assert lib.ibm_create(ctypes.byref(h), ctypes.byref(g), 0, 0) == _lib.IBM_E_ARG
    assert lib.ibm_levelset_prepare(None, None, None, None, None) == _lib.IBM_E_ARG
    assert lib.ibm_wall_stress(None, None, None, None, 0.0, None, None, None, None) == _lib.IBM_E_ARG
    assert lib.ibm_apply(None, None, None, None, 0.0, None, None, None) == _lib.IBM_E_ARG
    assert lib.ibm_destroy(None) == _lib.IBM_OK
