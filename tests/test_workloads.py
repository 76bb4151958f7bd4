"""Host checks of the seeded workload generators (shapes and counts only:
the generators hold none of the method's arithmetic)."""
import numpy as np

from paper_2502_10685_amd import workloads as W


def test_chain_zxz_shape_matches_the_stated_gate_count():
    wc = W.chain_zxz_circuit()
    assert wc.n == 4 and wc.m == 60200 and wc.n_params == 60000
    assert list(wc.op[:4]) == [W.CX] * 4
    assert list(zip(wc.q0[:4], wc.q1[:4])) == [(0, 1), (1, 2), (2, 3), (3, 0)]
    assert list(wc.op[4:7]) == [W.RZ, W.RX, W.RZ] and set(wc.q0[4:7]) == {0}
    rot = wc.op >= W.RX
    assert np.array_equal(wc.param[rot], np.arange(60000))
    assert np.all(wc.param[~rot] == -1)


def test_configs_are_seeded_and_reproducible():
    a, b = W.config3(count=8), W.config3(count=8)
    for x, y in zip(a, b):
        assert np.array_equal(x.op, y.op) and np.array_equal(x.theta, y.theta)
    assert W.config1().m == 160 and W.config4().n_params == 960


def test_spread_circuit_set_size_is_the_closed_form():
    """The oracle's final set of the spread circuit has 2^(n-k) 3^k strings and
    its <O> is the state vector's."""
    import oracle
    for n, k in ((6, 0), (6, 2), (8, 3), (9, 9)):
        w = W.spread_circuit(n + k, n, k)
        r = oracle.propagate(w)
        assert len(r.x) == w.meta["final_terms"] == 2 ** (n - k) * 3 ** k
        assert abs(r.expval - oracle.expval_sv(w)) <= 1e-12
