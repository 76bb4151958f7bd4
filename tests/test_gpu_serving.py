"""Serving loop: continuous batching with memory admission.  Every served
result must equal the same circuit's solo evaluation bit for bit, whatever
else is in flight, and agree with the state-vector oracle."""
import time

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


def _mix(count=40, seed=55, n_lo=4, n_hi=10, m_lo=200, m_hi=2500):
    reqs = []
    for i, (_, w) in enumerate(W.config5_requests(seed=seed, lam=1000.0, count=count, n_lo=n_lo, n_hi=n_hi,
                                                  m_lo=m_lo, m_hi=m_hi)):
        reqs.append(w)
    return reqs


def _wait(server, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = server.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "serving did not finish"
        time.sleep(0.001)
    return out


def test_served_equals_solo_bitwise(api):
    import torch
    ws = _mix()
    print(f"serving {len(ws)} requests", flush=True)
    solo = []
    for w in ws:
        c = api.Circuit.from_workload(w)
        solo.append(float(c.evaluate().item()))
        c.close()
    torch.cuda.synchronize()
    srv = api.Server(mem_budget_bytes=1 << 30, max_active=16)
    circs = [api.Circuit.from_workload(w) for w in ws]
    tickets = []
    for i, c in enumerate(circs):
        tickets.append(srv.submit(c))
        if i % 5 == 4:
            time.sleep(0.002)  # later requests arrive while earlier ones run
    res = _wait(srv, tickets)
    got = [res[t][0] for t in tickets]
    assert got == solo
    cnt = srv.counters()
    print(f"serving counters {cnt}", flush=True)
    assert cnt["max_in_flight"] > 1 and cnt["tile_launches"] > 0
    for w, v in zip(ws[:8], got):
        assert abs(v - oracle.expval_sv(w)) <= 1e-12
    srv.close()


def test_memory_budget_limits_in_flight(api):
    """A budget of one n = 10 weight array (8 MiB) admits the n = 10 requests
    one at a time; results are unchanged."""
    ws = [W.random_circuit(900 + i, 10, 400, W.obs_z(10, [0, 1])) for i in range(4)]
    solo = []
    for w in ws:
        c = api.Circuit.from_workload(w)
        solo.append(float(c.evaluate().item()))
    srv = api.Server(mem_budget_bytes=8 << 20, max_active=8)
    circs = [api.Circuit.from_workload(w) for w in ws]
    tickets = [srv.submit(c) for c in circs]
    res = _wait(srv, tickets)
    assert [res[t][0] for t in tickets] == solo
    assert srv.counters()["max_in_flight"] == 1
    from paper_2502_10685_amd._lib import PauliPropError
    big = api.Circuit.from_workload(W.random_circuit(3, 11, 50))
    with pytest.raises(PauliPropError):
        srv.submit(big)  # 4^11 * 8 bytes > budget
    srv.close()


def test_alone_vs_mix_same_request(api):
    """One request served alone, then again in the middle of a stream of
    others: identical bits."""
    target = W.random_circuit(4242, 9, 1500, W.obs_z(9, [0, 1]))
    srv = api.Server(mem_budget_bytes=1 << 30, max_active=32)
    t = srv.submit(api.Circuit.from_workload(target))
    alone = _wait(srv, [t])[t][0]
    others = [api.Circuit.from_workload(w) for w in _mix(count=20, seed=77)]
    ts = [srv.submit(c) for c in others[:10]]
    t2 = srv.submit(api.Circuit.from_workload(target))
    ts += [srv.submit(c) for c in others[10:]]
    res = _wait(srv, ts + [t2])
    assert res[t2][0] == alone
    assert abs(alone - oracle.expval_sv(target)) <= 1e-12
    srv.drain()
    srv.close()
