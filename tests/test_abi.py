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
