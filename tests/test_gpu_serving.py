"""Serving loop: continuous batching with memory admission.  Every served
result must equal the same circuit's solo evaluation bit for bit, whatever
else is in flight, and agree with the state-vector oracle."""
import math
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


def _config5_shape_requests():
    """Requests of the serving workload's shape (n ~ U{4..12}, m log-uniform
    in [1k, 60k]), seeded, with n = 11 and n = 12 ones forced in: one n = 12
    request with m >= 20k, n = 11 and n = 12 requests with m in the
    thousands, and a spread of smaller ones."""
    reqs = [w for _, w in W.config5_requests(seed=505, lam=1000.0, count=10, n_lo=4, n_hi=10, m_lo=1000,
                                             m_hi=8000)]
    rng = np.random.default_rng(5050)
    reqs.append(W.random_circuit(rng, 12, 21000, W.obs_random_2local(rng, 12)))
    reqs.append(W.random_circuit(rng, 12, 3500, W.obs_z(12, [0])))
    reqs.append(W.random_circuit(rng, 11, 6000, W.obs_random_2local(rng, 11)))
    reqs.append(W.random_circuit(rng, 11, 1200, W.obs_z(11, [0])))
    return reqs


def test_config5_shape_served_parity(api):
    """Every served <O> equals its solo pp_evaluate bit for bit and the FP64
    state vector within 1e-12, at the serving workload's sizes (n = 11 and
    n = 12 requests among smaller ones, one n = 12 request of 21,000 gates)."""
    import torch
    ws = _config5_shape_requests()
    print("config5-shape serving: " + ", ".join(f"n={w.n} m={w.m}" for w in ws), flush=True)
    solo = []
    for w in ws:
        c = api.Circuit.from_workload(w)
        solo.append(float(c.evaluate().item()))
        c.close()
    torch.cuda.synchronize()
    srv = api.Server(mem_budget_bytes=1 << 30, max_active=8)
    circs = [api.Circuit.from_workload(w) for w in ws]
    tickets = [srv.submit(c) for c in circs]
    res = _wait(srv, tickets, timeout=300.0)
    got = [res[t][0] for t in tickets]
    assert got == solo
    worst = 0.0
    for w, v in zip(ws, got):
        err = abs(v - oracle.expval_sv(w))
        worst = max(worst, err)
        assert err <= 1e-12, (w.name, w.n, w.m, v, err)
    print(f"config5-shape serving: max |served - state vector| = {worst:.2e}", flush=True)
    held, peak = srv.pool_bytes()
    assert peak <= 1 << 30
    srv.close()


def test_resubmit_with_new_theta(api):
    """A circuit served, then given new angles (on the caller's stream) and
    submitted again, is served at the new angles: the server orders its work
    after the upload.  Tiled and LDS-resident, host and device angles."""
    import torch
    rng = np.random.default_rng(606)
    srv = api.Server(mem_budget_bytes=1 << 30, max_active=8)
    for n, m in ((9, 2500), (6, 3000)):
        w = W.random_circuit(rng, n, m, W.obs_z(n, [0, 1]))
        served = api.Circuit.from_workload(w)
        solo = api.Circuit.from_workload(w)
        for rep in range(3):
            th = rng.uniform(0, 2 * math.pi, size=w.n_params)
            solo.set_theta(th)
            want = float(solo.evaluate().item())
            if rep % 2:
                served.set_theta(torch.tensor(th, device="cuda"))
            else:
                served.set_theta(th)
            t = srv.submit(served)
            got = _wait(srv, [t])[t][0]
            assert got == want, (n, rep, got, want)
            assert abs(got - oracle.expval_sv(w.with_theta(th))) <= 1e-12
    srv.close()


def test_duplicate_circuits_rejected(api):
    """One circuit twice in a batch, or submitted again before it is done, is
    an error (it would share one weight array between two evaluations)."""
    from paper_2502_10685_amd._lib import PauliPropError, PP_ERR_INVALID
    w = W.random_circuit(707, 9, 3000, W.obs_z(9, [0]))
    c = api.Circuit.from_workload(w)
    other = api.Circuit.from_workload(W.random_circuit(708, 8, 500))
    with pytest.raises(PauliPropError) as ei:
        api.evaluate_batch([c, other, c])
    assert ei.value.status == PP_ERR_INVALID
    srv = api.Server(mem_budget_bytes=1 << 30, max_active=4)
    t = srv.submit(c)
    with pytest.raises(PauliPropError) as ei:
        srv.submit(c)
    assert ei.value.status == PP_ERR_INVALID
    first = _wait(srv, [t])[t][0]
    t2 = srv.submit(c)  # done: may be submitted again
    assert _wait(srv, [t2])[t2][0] == first
    srv.close()


def test_queue_limit_returns_busy(api):
    """With a queue limit, submissions beyond it give PP_ERR_BUSY and queue
    nothing; the admitted ones finish with their solo results."""
    from paper_2502_10685_amd._lib import PauliPropError, PP_ERR_BUSY
    ws = [W.random_circuit(810 + i, 10, 4000, W.obs_z(10, [0, 1])) for i in range(6)]
    solo = []
    for w in ws:
        c = api.Circuit.from_workload(w)
        solo.append(float(c.evaluate().item()))
    srv = api.Server(mem_budget_bytes=8 << 20, max_active=1)
    srv.set_queue_limit(2)
    circs = [api.Circuit.from_workload(w) for w in ws]
    accepted, busy = {}, 0
    for i, c in enumerate(circs):
        try:
            accepted[srv.submit(c)] = i
        except PauliPropError as e:
            assert e.status == PP_ERR_BUSY
            busy += 1
    assert busy >= 1 and len(accepted) >= 2
    res = _wait(srv, list(accepted))
    for t, i in accepted.items():
        assert res[t][0] == solo[i]
    srv.close()


def test_pool_bounds_served_weights(api):
    """Served tiled requests run in the server's pool: the pool never holds
    more than the budget, and the library's device memory does not grow by
    one 4^n array per served circuit."""
    import torch
    from paper_2502_10685_amd._lib import memory_in_use
    ws = [W.random_circuit(900 + i, 10, 800, W.obs_z(10, [0, 1])) for i in range(12)]
    budget = 2 * (4 ** 10) * 8  # two n = 10 weight arrays
    srv = api.Server(mem_budget_bytes=budget, max_active=8)
    circs = [api.Circuit.from_workload(w) for w in ws]
    torch.cuda.synchronize()
    before, _ = memory_in_use()
    tickets = [srv.submit(c) for c in circs]
    res = _wait(srv, tickets)
    after, _ = memory_in_use()
    held, peak = srv.pool_bytes()
    assert peak <= budget and held <= budget
    assert srv.counters()["max_in_flight"] <= 2
    # 12 circuits x 8 MiB would be 96 MiB; schedules and the pool are far less
    assert after - before <= budget + (8 << 20), (before, after)
    for w, t in zip(ws[:3], tickets[:3]):
        assert abs(res[t][0] - oracle.expval_sv(w)) <= 1e-12
    srv.close()
