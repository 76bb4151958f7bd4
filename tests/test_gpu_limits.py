"""Largest and boundary sizes of both engines against the oracle: the
largest DENSE register (n = 16, 4^16 FP64 weights = 32 GiB, where the tile
passes use 64-bit offsets), the AUTO boundary (n = 13 dense, n = 14
SPARSE), and the largest SPARSE register (n = 64, 128-bit keys, sort-merge)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_dense_largest_register_n16(api):
    """n = 16 in FP64: every tile pass streams 4^16 weights (32 GiB); a short
    random circuit, checked against the state vector and, string by string,
    against the scalar propagator."""
    rng = np.random.default_rng(1600)
    wc = W.random_circuit(rng, 16, 70, W.obs_z(16, [0, 15]))
    _say("dense n=16 m=70")
    want = oracle.propagate(wc, cap=1 << 20)
    c = api.Circuit.from_workload(wc, engine="dense")
    ev = float(c.evaluate().item())
    _say(f"dense n=16: <O> = {ev!r}, passes {c.stats()['passes']}")
    assert abs(ev - oracle.expval_sv(wc)) <= TOL64
    assert abs(ev - want.expval) <= TOL64
    # an untracked dense run reports the strings of nonzero weight: a subset
    # of the structural set holding every string not (near) zero
    x, z, v = c.terms(capacity=1 << 20)
    got = {(int(a), int(b)): float(w) for a, b, w in zip(x, z, v)}
    ref = {(int(a), int(b)): float(w) for a, b, w in zip(want.x, want.z, want.c)}
    assert set(got) <= set(ref)
    assert all(key in got for key, w in ref.items() if abs(w) > 1e-9)
    assert max(abs(w - got.get(key, 0.0)) for key, w in ref.items()) <= TOL64
    c.close()


@pytest.mark.parametrize("n,engine_code", [(13, 1), (14, 2)])
def test_auto_engine_boundary(api, n, engine_code):
    """AUTO picks DENSE up to n = 13 and SPARSE from n = 14 on; both match the
    state vector."""
    rng = np.random.default_rng(1300 + n)
    wc = W.random_circuit(rng, n, 150, W.obs_tfim(n))
    _say(f"auto engine n={n}")
    c = api.Circuit.from_workload(wc, engine="auto", max_terms=1 << 22)
    ev = float(c.evaluate().item())
    assert c.stats()["engine"] == engine_code
    assert abs(ev - oracle.expval_sv(wc)) <= TOL64
    c.close()


def test_sparse_largest_register_n64(api):
    """n = 64: keys fill both 64-bit words (the sort-merge engine; the frame
    engine stops at n = 31).  The observable touches qubits 0 and 63; strings,
    weights and U equal the scalar propagator's."""
    rng = np.random.default_rng(6400)
    wc = W.random_circuit(rng, 64, 90, W.obs_z(64, [0, 63]))
    _say("sparse n=64 m=90")
    want = oracle.propagate(wc, cap=1 << 20)
    c = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 20)
    ev = float(c.evaluate().item())
    st = c.stats()
    assert not st["overflow"]
    assert abs(ev - want.expval) <= TOL64
    x, z, v = c.terms(capacity=1 << 20)
    assert np.array_equal(x, want.x) and np.array_equal(z, want.z)
    assert float(np.max(np.abs(v - want.c))) <= TOL64
    assert st["term_updates"] == want.updates
    c.close()
