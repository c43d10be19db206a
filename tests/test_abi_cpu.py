"""CPU-side checks of the C ABI: the shared library loads without a GPU and
exports every function that include/hyperion_mi355x.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperion_mi355x.h")
LIB = os.path.join(ROOT, "paper_2604_01176_amd", "libhyperion_mi355x.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hyp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared_functions()
    for required in ["hyp_build_hamiltonian", "hyp_apply_h", "hyp_expectation",
                     "hyp_pool_gradients", "hyp_apply_excitation", "hyp_sector_create",
                     "hyp_sector_destroy", "hyp_ham_destroy", "hyp_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("library not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2604_01176_amd import _lib
    names = declared_functions()
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def test_last_error_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.hyp_last_error.restype = ctypes.c_char_p
    lib.hyp_sector_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    # argument validation happens before any device call
    assert lib.hyp_sector_create(17, 1, 1, None) == 1  # NULL out -> HYP_ERR_ARG
    out = ctypes.c_void_p()
    assert lib.hyp_sector_create(17, 1, 1, ctypes.byref(out)) == 2  # n_orb > 16 -> HYP_ERR_SECTOR
    assert b"n_orb" in lib.hyp_last_error()
    assert lib.hyp_sector_create(4, 5, 1, ctypes.byref(out)) == 2


def test_switch_argument_checks_without_gpu():
    """The process-wide switches validate their argument before any device
    call (HYP_ERR_ARG = 1), and accept every documented value."""
    lib = ctypes.CDLL(LIB)
    cases = (("hyp_set_same_spin_cores", (0, 1, 2), (-1, 3), 2),
             ("hyp_set_mixed_matrix_cores", (0, 1, 2), (-1, 3), 2),
             ("hyp_set_same_spin_groups", (0, 1, 2, 4), (-1, 3, 8), 2),
             ("hyp_set_row_staging", (0, 1), (-1, 2), 0),
             ("hyp_set_support_skip", (0, 1), (-1, 2), 1))
    for name, good, bad, default in cases:
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int]
        for v in bad:
            assert f(v) == 1, (name, v)
        for v in good:
            assert f(v) == 0, (name, v)
        assert f(default) == 0
