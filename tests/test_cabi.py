"""The C-ABI library loads on the CPU host and exports every function its headers declare (no GPU
calls). Also checks host-side argument validation that returns before any launch."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_21697_amd", "libtdde.so")


def _declared():
    names = []
    for h in ("tdde.h", "tdde_mlp.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(tdde_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2512_21697_amd.build import build
        build()
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_match_header():
    from paper_2512_21697_amd import _lib
    names = set(_declared())
    for n in _lib.EXPORTS:
        assert n in names


def test_create_rejects_bad_dims_without_gpu(lib):
    class Dims(C.Structure):
        _fields_ = [("nr", C.c_int32), ("nang", C.c_int32), ("half_band", C.c_int32), ("batch", C.c_int32),
                    ("n_fields", C.c_int32)]
    lib.tdde_create.restype = C.c_int
    lib.tdde_last_error.restype = C.c_char_p
    h = C.c_void_p()
    assert lib.tdde_create(C.byref(Dims(0, 4, 6, 1, 1)), None, C.byref(h)) == -1
    assert b"dims" in lib.tdde_last_error(None)
    assert lib.tdde_create(C.byref(Dims(10, 4, 9, 1, 1)), None, C.byref(h)) == -1
    ok = lib.tdde_create(C.byref(Dims(10, 4, 6, 1, 1)), None, C.byref(h))
    assert ok == 0
    lib.tdde_destroy.restype = C.c_int
    assert lib.tdde_destroy(h) == 0


def test_status_strings(lib):
    lib.tdde_status_string.restype = C.c_char_p
    assert lib.tdde_status_string(0) == b"ok"
    assert lib.tdde_status_string(1) == b"not converged"
    lib.tdde_mlp_param_count.restype = C.c_int64
    assert lib.tdde_mlp_param_count() == 256 * 32 + 256 + 256 * 256 + 256 + 512 + 2
