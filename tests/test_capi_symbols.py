"""The C-ABI library loads and exports every symbol include/pauliprop.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pauliprop.h")
LIB = os.path.join(ROOT, "paper_2502_10685_amd", "libpauliprop.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^PP_API\s+[\w\s\*]*?\b(pp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_api():
    names = declared_symbols()
    for want in ("pp_circuit_create", "pp_circuit_load_gates", "pp_circuit_set_theta",
                 "pp_circuit_set_observable", "pp_evaluate", "pp_evaluate_batch", "pp_gradient",
                 "pp_get_terms", "pp_get_stats", "pp_circuit_destroy"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpauliprop.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpauliprop.so not built")
def test_version_and_null_safety_without_gpu():
    from paper_2502_10685_amd import _lib as L
    lib = L.load()
    assert lib.pp_version().startswith(b"pauliprop")
    lib.pp_circuit_destroy(None)  # NULL-safe
    st = L.PPStats()
    assert lib.pp_get_stats(None, ctypes.byref(st)) == L.PP_ERR_INVALID
    assert lib.pp_circuit_create(4, 0, 0, None) == L.PP_ERR_INVALID
    h = ctypes.c_void_p()
    assert lib.pp_circuit_create(0, 0, 0, ctypes.byref(h)) == L.PP_ERR_INVALID
    assert lib.pp_circuit_create(65, 0, 0, ctypes.byref(h)) == L.PP_ERR_INVALID
    assert lib.pp_circuit_create(4, 7, 0, ctypes.byref(h)) == L.PP_ERR_INVALID
    assert b"dtype" in lib.pp_last_error()


def test_stats_struct_layout_matches_header():
    from paper_2502_10685_amd import _lib as L
    assert ctypes.sizeof(L.PPStats) == 7 * 8 + 4 * 4
