"""Truncated propagation on the sparse engine (approximate, outside the
exact method): a dropped string of weight w moves <O> by at most |w|, since
|<psi|P|psi>| <= 1 for every Pauli string P, so the summed dropped weight
bounds the error.  Checks: the no-op settings reproduce the exact run bit for
bit; the cuts hold on the final set; |<O>_trunc - <O>_exact| <= dropped
(+ 1e-12 rounding), with <O>_exact from the oracle's state vector.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _weights(x, z):
    return np.array([bin(int(a) | int(b)).count("1") for a, b in zip(x, z)], dtype=np.int64)


def test_noop_truncation_is_the_exact_run(api):
    wc = W.random_circuit(np.random.default_rng(3), 10, 200, W.obs_z(10, [0, 1]))
    _say("truncation no-op n=10")
    a = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 21)
    ea = float(a.evaluate().item())
    xa, za, ca = a.terms(capacity=1 << 21)
    b = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 21)
    b.set_truncation(0.0, 64)
    eb = float(b.evaluate().item())
    xb, zb, cb = b.terms(capacity=1 << 21)
    assert ea == eb
    assert np.array_equal(xa, xb) and np.array_equal(za, zb)
    assert np.array_equal(ca.view(np.uint64), cb.view(np.uint64))
    assert b.truncation_dropped() == 0.0
    a.close()
    b.close()


@pytest.mark.parametrize("eps,wmax", [(0.0, 3), (1e-3, 64), (1e-4, 5)])
def test_truncation_respects_cuts_and_error_bound(api, eps, wmax):
    n = 12
    wc = W.random_circuit(np.random.default_rng(12), n, 260, W.obs_z(n, [0, 1]))
    _say(f"truncation n={n} eps={eps} max_weight={wmax}")
    exact = oracle.expval_sv(wc)
    c = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 23)
    c.set_truncation(eps, wmax)
    ev = float(c.evaluate().item())
    dropped = c.truncation_dropped()
    x, z, v = c.terms(capacity=1 << 23)
    assert dropped > 0.0
    assert len(x) > 0 and int(_weights(x, z).max()) <= wmax
    assert float(np.min(np.abs(v))) >= eps
    assert abs(ev - exact) <= dropped + 1e-12, (ev, exact, dropped)
    c.close()


def test_truncation_beyond_dense_range(api):
    """n = 22: weight-truncated propagation of a 200-gate circuit; the state
    vector (4M amplitudes) still gives the exact value."""
    n = 22
    wc = W.random_circuit(np.random.default_rng(22), n, 200, W.obs_z(n, [0, 1]))
    _say(f"truncation n={n}")
    exact = oracle.expval_sv(wc)
    c = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 22)
    c.set_truncation(1e-5, 6)
    ev = float(c.evaluate().item())
    st = c.stats()
    assert not st["overflow"]
    assert abs(ev - exact) <= c.truncation_dropped() + 1e-12
    c.close()


def test_truncation_rejects_bad_arguments(api):
    from paper_2502_10685_amd import _lib as L
    wc = W.random_circuit(np.random.default_rng(1), 6, 50)
    d = api.Circuit.from_workload(wc, engine="dense")
    with pytest.raises(L.PauliPropError):
        d.set_truncation(1e-3, 4)
    d.close()
    s = api.Circuit.from_workload(wc, engine="sparse")
    with pytest.raises(L.PauliPropError):
        s.set_truncation(-1.0, 4)
    with pytest.raises(L.PauliPropError):
        s.set_truncation(0.0, 0)
    with pytest.raises(L.PauliPropError):
        s.truncation_dropped()
    s.close()
