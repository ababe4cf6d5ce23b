"""The C-ABI library loads and exports every function that include/aci.h
declares (no device calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_00037_amd", "libaci.so")
HDR = os.path.join(ROOT, "include", "aci.h")


def declared_functions():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(aci_\w+)\s*\(", src, re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("aci_ctx_create", "aci_elementwise", "aci_prrlu", "aci_pi_eval",
              "aci_env_contract", "aci_gather", "aci_result_free", "aci_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libaci.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libaci.so not built")
def test_binding_matches_exports():
    from paper_2604_00037_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_null_context_is_rejected_without_device():
    if not os.path.exists(LIB):
        pytest.skip("libaci.so not built")
    lib = ctypes.CDLL(LIB)
    lib.aci_prrlu.restype = ctypes.c_int
    # a null context is an argument error, reported before any device call
    assert lib.aci_prrlu(None, 0, None, 1, 1, 1, ctypes.c_double(0.0), 1, 0,
                         None, None, None, None, None, 1) == -1
    lib.aci_last_error.restype = ctypes.c_char_p
    assert lib.aci_last_error(None) == b"null context"
