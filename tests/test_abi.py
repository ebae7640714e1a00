"""CPU checks of the C ABI: the library builds for gfx950, loads, and exports
every function that include/sj.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            src = re.sub(r"//[^\n]*", "", src)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s+\**(sj_[a-z_0-9]+)\s*\(",
                                src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1908_11740_amd import build
    path = build.build(force=False)
    return ctypes.CDLL(path)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("sj_partition", "sj_join", "sj_join_count", "sj_part_free", "sj_status_string"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_without_gpu(lib):
    lib.sj_status_string.restype = ctypes.c_char_p
    for code in range(-7, 1):
        assert lib.sj_status_string(code)
    lib.sj_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.sj_version()


def test_library_targets_gfx950():
    from paper_1908_11740_amd import build
    data = open(build.LIB, "rb").read()
    assert b"gfx950" in data
