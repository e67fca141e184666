"""The C ABI library loads and exports every function include/mi_knn.h
declares; the Python binding covers the same names.  No device calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi_knn.h")
LIB = os.path.join(ROOT, "paper_1702_08734_amd", "libmiknn.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mk_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libhandle():
    if not os.path.exists(LIB):
        from paper_1702_08734_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("mk_knn_search", "mk_kselect", "mk_ivfpq_train", "mk_ivfpq_add",
              "mk_ivfpq_search", "mk_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(libhandle):
    missing = [n for n in declared() if not hasattr(libhandle, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1702_08734_amd import api
    assert sorted(api._SIGS) == declared()


def test_argument_errors_need_no_device(libhandle):
    # validation happens before any HIP call
    libhandle.mk_knn_search.restype = ctypes.c_int32
    vp = ctypes.c_void_p
    libhandle.mk_knn_search.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    assert libhandle.mk_knn_search(None, 1, None, 1, 4, 2000, 0, None, None, None) == -2
    assert libhandle.mk_knn_search(None, 1, None, 1, 4, 0, 0, None, None, None) == -1
    assert libhandle.mk_knn_search(None, 0, None, 1, 4, 5, 0, None, None, None) == 0
    libhandle.mk_last_error.restype = ctypes.c_char_p
    libhandle.mk_knn_search(None, 1, None, 1, 0, 5, 0, None, None, None)
    assert b"d must be" in libhandle.mk_last_error()


def test_bad_files_refused_without_a_device(libhandle, tmp_path):
    # the header is checked before any HIP call
    import ctypes as C
    vp = C.c_void_p
    for fn in ("mk_ivfpq_load", "mk_mlp_load"):
        f = getattr(libhandle, fn)
        f.restype = C.c_int32
        f.argtypes = [C.c_char_p, C.POINTER(vp)]
        out = vp(1)
        missing = str(tmp_path / "none.bin").encode()
        assert f(missing, C.byref(out)) == -1 and not out.value
        junk = tmp_path / "junk.bin"
        junk.write_bytes(b"not an index or network file at all")
        out = vp(1)
        assert f(str(junk).encode(), C.byref(out)) == -1 and not out.value
