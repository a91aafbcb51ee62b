"""The C-ABI library loads and exports every entry point include/vj.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vj.h")
LIB = os.path.join(ROOT, "paper_2603_16360_amd", "libvj.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vj_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("vj_build_merged_index", "vj_join", "vj_bruteforce_join",
                 "vj_pairs_export", "vj_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import pytest
        pytest.skip("libvj.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    import pytest
    if not os.path.exists(LIB):
        pytest.skip("libvj.so not built")
    from paper_2603_16360_amd import vj
    assert set(declared()) == set(vj.EXPORTED)


def test_last_error_is_empty_string_initially():
    import pytest
    if not os.path.exists(LIB):
        pytest.skip("libvj.so not built")
    lib = ctypes.CDLL(LIB)
    lib.vj_last_error.restype = ctypes.c_char_p
    assert lib.vj_last_error() == b""


def test_index_size_limit_is_checked_before_any_device_work():
    # node ids of an index must stay below 2^30; the check runs before any
    # HIP call, so it needs no GPU (the pointers are never read)
    import pytest
    if not os.path.exists(LIB):
        pytest.skip("libvj.so not built")
    lib = ctypes.CDLL(LIB)
    lib.vj_last_error.restype = ctypes.c_char_p
    f = lib.vj_build_merged_index
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                  ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)
    st = f(fake, 1 << 29, fake, 1 << 29, 16, 0, None, None, ctypes.byref(out))
    assert st == 6 and b"2^30" in lib.vj_last_error()
    assert out.value is None
    # d out of range and a null vector pointer are argument errors too
    assert f(fake, 4, fake, 4, 0, 0, None, None, ctypes.byref(out)) == 1
    assert f(fake, 4, None, 4, 8, 0, None, None, ctypes.byref(out)) == 1
