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
    # entry points of the density matrix and of truncation reject NULL first
    assert lib.pp_density_matrix(None, None, None) == L.PP_ERR_INVALID
    assert lib.pp_circuit_set_truncation(None, 0.0, 4) == L.PP_ERR_INVALID
    v = ctypes.c_double(0.0)
    assert lib.pp_get_truncation(None, None, ctypes.byref(v)) == L.PP_ERR_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpauliprop.so not built")
def test_boundary_entry_points_reject_bad_arguments_without_gpu():
    """Allocator hook, memory query, parameter-shift gradient and the serving
    controls validate their arguments before touching a device."""
    from paper_2502_10685_amd import _lib as L
    lib = L.load()
    half = L.PPAllocator(L.ALLOC_FN(lambda n, s, u: None), ctypes.cast(None, L.FREE_FN), None)
    assert lib.pp_set_allocator(ctypes.byref(half)) == L.PP_ERR_INVALID
    assert b"alloc and free" in lib.pp_last_error()
    assert lib.pp_set_allocator(None) == L.PP_OK  # the default pool
    b, n = ctypes.c_int64(-1), ctypes.c_int64(-1)
    assert lib.pp_memory_in_use(ctypes.byref(b), ctypes.byref(n)) == L.PP_OK
    assert b.value >= 0 and n.value >= 0
    assert lib.pp_memory_in_use(None, None) == L.PP_ERR_INVALID
    assert lib.pp_psr_gradient(None, None, None) == L.PP_ERR_INVALID
    assert lib.pp_server_set_queue_limit(None, 4) == L.PP_ERR_INVALID
    assert lib.pp_server_pool_bytes(None, None, None) == L.PP_ERR_INVALID
    t = ctypes.c_int64(0)
    assert lib.pp_server_submit(None, None, ctypes.byref(t)) == L.PP_ERR_INVALID
    assert lib.pp_evaluate_batch(None, -1, None, None) == L.PP_ERR_INVALID
    lib.pp_server_destroy(None)  # NULL-safe


def test_stats_struct_layout_matches_header():
    from paper_2502_10685_amd import _lib as L
    assert ctypes.sizeof(L.PPStats) == 7 * 8 + 4 * 4


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpauliprop.so not built")
def test_planner_host_logic():
    """The DENSE scheduler, run on the host: one pass when the tile is the
    whole register, every op counted once, composition only merges
    single-qubit gates, tracked schedules keep one op per gate."""
    import numpy as np
    from paper_2502_10685_amd import _lib as L
    from paper_2502_10685_amd import workloads as W
    rng = np.random.default_rng(4)
    w = W.random_circuit(rng, 9, 3000)
    ncx = int(np.sum(w.op == 2))
    ops, passes = L.plan_dense_info(9, w.op, w.q0, w.q1, w.param, w.n_params, 9)
    assert passes == 1 and ncx < ops < w.m
    ops_t, passes_t, per = L.plan_dense_info(9, w.op, w.q0, w.q1, w.param, w.n_params, 5, compose=False,
                                             reorder=False, want_passes=True)
    assert ops_t == w.m and per.sum() == w.m and len(per) == passes_t
    ops_c, passes_c, per_c = L.plan_dense_info(9, w.op, w.q0, w.q1, w.param, w.n_params, 5, want_passes=True)
    assert per_c.sum() == ops_c and ops_c < ops_t
    assert passes_c < passes_t  # reordering packs more gates per tile pass
    hea = W.config4()
    ops_h, passes_h = L.plan_dense_info(8, hea.op, hea.q0, hea.q1, hea.param, hea.n_params, 8)
    # per layer: 8 wires x (RX RY RZ) fold into 8 U1 ops, plus 8 CX
    assert ops_h == 40 * 16
    with pytest.raises(L.PauliPropError):
        L.plan_dense_info(9, w.op, w.q0 + 20, w.q1, w.param, w.n_params, 5)
    with pytest.raises(L.PauliPropError):
        L.plan_dense_info(9, w.op, w.q0, w.q1, w.param, w.n_params, 3)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpauliprop.so not built")
@pytest.mark.parametrize("n", list(range(1, 13)))
def test_planner_self_check_random(n):
    """The planner's structural self-check holds for random circuits of every
    size, for LDS-resident schedules and every tile size."""
    import numpy as np
    from paper_2502_10685_amd import _lib as L
    from paper_2502_10685_amd import workloads as W
    rng = np.random.default_rng(700 + n)
    for rep in range(3):
        w = W.random_circuit(rng, n, int(rng.integers(1, 1500)))
        ks = [n] + [k for k in (4, 5, 6, 7) if k < n]
        for k in ks:
            for compose in (True, False):
                ops, passes = L.plan_dense_info(n, w.op, w.q0, w.q1, w.param, w.n_params, k, compose=compose,
                                                reorder=compose)
                assert ops >= 1 and passes >= 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpauliprop.so not built")
def test_tuning_knobs_validate_without_gpu():
    """pp_tune_set / pp_tune_get only touch host tables: every key accepts its
    documented range and rejects the rest (PP_ERR_INVALID = 1)."""
    from paper_2502_10685_amd import _lib as L
    lib = L.load()
    v = ctypes.c_int32(-1)
    for cls in range(3):
        old = L.tune_get(L.PP_TUNE_SORT_SHAPE, cls)
        assert old == 0  # default shape: 8 key bits per pass, 8 terms per thread
        for shape in range(6):
            assert lib.pp_tune_set(L.PP_TUNE_SORT_SHAPE, cls, shape) == 0
            assert lib.pp_tune_get(L.PP_TUNE_SORT_SHAPE, cls, ctypes.byref(v)) == 0 and v.value == shape
        L.tune_set(L.PP_TUNE_SORT_SHAPE, cls, old)
    for bad in ((-1, 0), (3, 0), (0, -1), (0, 6)):
        assert lib.pp_tune_set(L.PP_TUNE_SORT_SHAPE, *bad) == 1
    assert lib.pp_tune_get(L.PP_TUNE_SORT_SHAPE, 3, ctypes.byref(v)) == 1
    assert lib.pp_tune_set(L.PP_TUNE_TILE_KERNEL, 7, 2) == 1  # wave-per-tile needs k <= 6
    assert lib.pp_tune_set(L.PP_TUNE_RESIDENT_BLOCK, 6, 300) == 1
    assert lib.pp_tune_set(99, 0, 0) == 1
