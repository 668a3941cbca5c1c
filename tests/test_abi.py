"""The C ABI library loads on the CPU and exports every entry point that
include/mbh.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbh.h")
LIB = os.path.join(ROOT, "paper_2111_01064_amd", "libmbh.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbh_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_three_likelihood_entry_points():
    names = declared_functions()
    for n in ("mbh_build_reference_coeffs", "mbh_loglike_heterodyned", "mbh_loglike_full"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbh.so not built")
def test_error_strings_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.mbh_strerror.restype = ctypes.c_char_p
    lib.mbh_strerror.argtypes = [ctypes.c_int32]
    assert lib.mbh_strerror(-3).decode().startswith("reference")
    lib.mbh_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.mbh_last_error(), bytes)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbh.so not built")
def test_binding_declares_every_entry_point():
    """The Python binding gives every declared entry point an argument list
    (the two string functions are typed where the errors are raised)."""
    from paper_2111_01064_amd import mbh

    missing = [n for n in declared_functions()
               if n not in mbh._SIGS and n not in ("mbh_last_error", "mbh_strerror")]
    assert not missing, missing
    extra = [n for n in mbh._SIGS if n not in declared_functions()]
    assert not extra, extra


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmbh.so not built")
def test_binding_argument_counts_match_the_header():
    """Each binding's argument list has as many entries as the declaration
    has parameters (a dropped or added argument would shift every later one)."""
    from paper_2111_01064_amd import mbh

    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    checked = 0
    for m in re.finditer(r"\b(?:mbh_status|const char \*|void)\s+(mbh_\w+)\s*\(([^;{]*?)\)\s*;", src, re.S):
        name, params = m.group(1), m.group(2).strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        if name in mbh._SIGS:
            assert len(mbh._SIGS[name]) == n, (name, n, len(mbh._SIGS[name]))
            checked += 1
    assert checked >= 50
