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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libaci.so not built")
@pytest.mark.parametrize("R,ndim", [(1, 1), (4, 1), (3, 2), (2, 3), (5, 3)])
def test_host_stencil_builder_matches_the_oracle(R, ndim):
    """aci_mpo_stencil is host logic: its cores equal the oracle's,
    entry for entry, for every axis (both written from the carry rule)."""
    import numpy as np
    from oracle import timestep as T
    lib = ctypes.CDLL(LIB)
    lib.aci_mpo_stencil.restype = ctypes.c_int
    L = R * ndim
    for axis in range(ndim):
        w = np.random.default_rng(10 * R + ndim + axis).standard_normal(3)
        cores = (ctypes.c_double * (36 * L))()
        ranks = (ctypes.c_int32 * (L + 1))()
        assert lib.aci_mpo_stencil(R, ndim, axis, (ctypes.c_double * 3)(*w), cores, ranks) == 0
        flat = np.ctypeslib.as_array(cores)
        ref = T.stencil_mpo(R, ndim, axis, w)
        for l in range(L):
            shape = (ranks[l], 2, 2, ranks[l + 1])
            assert shape == ref[l].shape
            assert np.array_equal(flat[36 * l:36 * l + int(np.prod(shape))].reshape(shape), ref[l])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libaci.so not built")
def test_host_stencil_builder_rejects_bad_arguments():
    lib = ctypes.CDLL(LIB)
    lib.aci_mpo_stencil.restype = ctypes.c_int
    w = (ctypes.c_double * 3)(1.0, -2.0, 1.0)
    cores = (ctypes.c_double * (36 * 200))()
    ranks = (ctypes.c_int32 * 201)()
    assert lib.aci_mpo_stencil(0, 1, 0, w, cores, ranks) == -1       # R < 1
    assert lib.aci_mpo_stencil(4, 2, 2, w, cores, ranks) == -1       # axis >= ndim
    assert lib.aci_mpo_stencil(4, 2, 0, None, cores, ranks) == -1
    assert lib.aci_mpo_stencil(65, 2, 0, w, cores, ranks) == -6      # L > ACI_MAX_SITES
