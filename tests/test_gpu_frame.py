"""The Clifford-frame SPARSE engine (default for exact runs with n <= 31)
against the sort-merge engine (PP_OPT_SPARSE_FRAME = 0) and the oracle: the
same string sets, the same term-update counts, weights equal to the last
bit (both round a merged weight as the sum of two rounded products), and
<O> within 1e-12 of the state vector."""
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(api, wc, frame, dtype="f64", cap=1 << 22):
    from paper_2502_10685_amd import _lib as L
    c = api.Circuit.from_workload(wc, engine="sparse", dtype=dtype, max_terms=cap)
    c.set_option(L.PP_OPT_SPARSE_FRAME, 1 if frame else 0)
    ev = float(c.evaluate().item())
    st = c.stats()
    x, z, v = c.terms(capacity=cap)
    c.close()
    return ev, st, x, z, v


@pytest.mark.parametrize("n,m,seed", [(6, 400, 1), (9, 250, 2), (14, 190, 3), (20, 200, 4)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_frame_equals_sort_merge(api, n, m, seed, dtype):
    wc = W.random_circuit(np.random.default_rng(600 + seed), n, m, W.obs_random_2local(np.random.default_rng(seed), n))
    _say(f"frame vs sort-merge n={n} m={m} {dtype}")
    ev_f, st_f, xf, zf, vf = _run(api, wc, True, dtype)
    ev_s, st_s, xs, zs, vs = _run(api, wc, False, dtype)
    assert st_f["final_terms"] == st_s["final_terms"] and st_f["term_updates"] == st_s["term_updates"]
    assert not st_f["overflow"]
    assert np.array_equal(xf, xs) and np.array_equal(zf, zs), "string sets differ"
    if dtype == "f64":
        assert np.array_equal(vf.view(np.uint64), vs.view(np.uint64)), float(np.max(np.abs(vf - vs)))
        assert abs(ev_f - ev_s) <= TOL64
        if n <= 14:
            assert abs(ev_f - oracle.expval_sv(wc)) <= TOL64
    else:
        assert float(np.max(np.abs(vf - vs))) <= TOL32
        assert abs(ev_f - ev_s) <= TOL32


def test_frame_matches_oracle_strings(api):
    """A Clifford-heavy circuit: the frame folds every Clifford gate into the
    rotation axes; the final strings (after the frame is applied) equal the
    scalar propagator's string for string."""
    rng = np.random.default_rng(640)
    wc = W.random_circuit(rng, 12, 160, W.obs_tfim(12))
    _say("frame vs oracle strings n=12")
    want = oracle.propagate(wc)
    ev, st, x, z, v = _run(api, wc, True)
    assert abs(ev - want.expval) <= TOL64
    assert np.array_equal(x, want.x) and np.array_equal(z, want.z)
    assert float(np.max(np.abs(v - want.c))) <= TOL64
    assert st["term_updates"] == want.updates


@pytest.mark.parametrize("n", [31, 32])
def test_frame_boundary_n31_n32(api, n):
    """n = 31 is the largest frame run (62 key bits), n = 32 takes the
    sort-merge engine; both match the oracle's strings (small sets)."""
    rng = np.random.default_rng(3100 + n)
    wc = W.random_circuit(rng, n, 120, W.obs_z(n, [0, n - 1]))
    _say(f"frame boundary n={n}")
    want = oracle.propagate(wc, cap=1 << 20)
    ev, st, x, z, v = _run(api, wc, True, cap=1 << 20)
    assert abs(ev - want.expval) <= TOL64
    assert np.array_equal(x, want.x) and np.array_equal(z, want.z)
    assert float(np.max(np.abs(v - want.c))) <= TOL64
    assert st["term_updates"] == want.updates


def test_frame_capacity_overflow(api):
    """More strings than the capacity: reported, <O> is NaN, terms refuse."""
    from paper_2502_10685_amd._lib import PauliPropError
    wc = W.random_circuit(np.random.default_rng(3), 10, 300, W.obs_z(10, [0]))
    c = api.Circuit.from_workload(wc, engine="sparse", max_terms=5000)
    ev = float(c.evaluate().item())
    assert c.stats()["overflow"] and np.isnan(ev)
    with pytest.raises(PauliPropError):
        c.terms(capacity=1 << 20)
    c.close()
