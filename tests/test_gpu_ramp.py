"""The ramp of a DENSE evaluation (PP_OPT_FRAME_RAMP): the last gates of the
Heisenberg sweep run in the Clifford frame while the string set is small,
then its strings move into the 4^n array for the rest.  Against the state
vector and the scalar propagator (FP64 1e-12, FP32 1e-5), against the plain
DENSE run, under graph replay, inside a batch and a server, and the entry
points that refuse it."""
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


@pytest.mark.parametrize("n,m,ramp,obs", [(8, 600, 4, "z"), (8, 600, 10, "tfim"), (6, 400, 3, "z"),
                                          (11, 500, 6, "z"), (9, 300, 2, "tfim")])
def test_ramp_matches_oracle_and_plain(api, n, m, ramp, obs):
    rng = np.random.default_rng(7000 + n + ramp)
    o = W.obs_z(n, [0, n - 1]) if obs == "z" else W.obs_tfim(n)
    wc = W.random_circuit(rng, n, m, o)
    _say(f"ramp n={n} m={m} t={ramp} obs={obs}")
    sv = oracle.expval_sv(wc)
    plain = api.Circuit.from_workload(wc, engine="dense")
    ev_p = float(plain.evaluate().item())
    c = api.Circuit.from_workload(wc, engine="dense", frame_ramp=ramp)
    ev = float(c.evaluate().item())
    assert abs(ev - sv) <= TOL64 and abs(ev - ev_p) <= TOL64
    assert c.stats()["passes"] >= plain.stats()["passes"]
    ev2 = float(c.evaluate().item())  # a second evaluation starts from the observable again
    assert ev2 == ev
    if 8 <= n <= 9:  # tiled: the final weights stay in the 4^n array (oracle strings up to n = 9)
        x, z, v = c.terms()
        want = oracle.propagate(wc)
        got = {(int(a), int(b)): float(w) for a, b, w in zip(x, z, v)}
        ref = {(int(a), int(b)): float(w) for a, b, w in zip(want.x, want.z, want.c)}
        assert set(got) <= set(ref)
        assert all(key in got for key, w in ref.items() if abs(w) > 1e-9)
        assert max(abs(w - got.get(key, 0.0)) for key, w in ref.items()) <= TOL64
    c.close()
    plain.close()


def test_ramp_fp32(api):
    wc = W.random_circuit(np.random.default_rng(7100), 9, 500, W.obs_z(9, [0, 1]))
    _say("ramp fp32 n=9")
    c = api.Circuit.from_workload(wc, engine="dense", dtype="f32", frame_ramp=6)
    assert abs(float(c.evaluate().item()) - oracle.expval_sv(wc)) <= TOL32
    c.close()


def test_ramp_edge_cases(api):
    """A Clifford-only circuit (the frame takes every gate), an observable
    larger than the ramp's limit (no ramp: the plain run), and a ramp limit
    above 4^n (the frame takes the whole circuit)."""
    n = 8
    rng = np.random.default_rng(7200)
    g, p = W.random_gates(rng, n, 200)
    cliff = np.asarray(g[0]) <= 2
    gates = tuple(np.asarray(a)[cliff] for a in g)
    wcl = W.make_circuit(n, (gates[0], gates[1], gates[2], np.full(int(cliff.sum()), -1, np.int32)), 0,
                         W.obs_tfim(n), [])
    _say("ramp clifford-only")
    c = api.Circuit.from_workload(wcl, engine="dense", frame_ramp=8)
    assert abs(float(c.evaluate().item()) - oracle.expval_sv(wcl)) <= TOL64
    c.close()
    wc = W.random_circuit(np.random.default_rng(7201), n, 300, W.obs_tfim(n))
    _say("ramp with an observable above its limit")
    c = api.Circuit.from_workload(wc, engine="dense", frame_ramp=14)  # limit 4 strings < 15 terms
    assert abs(float(c.evaluate().item()) - oracle.expval_sv(wc)) <= TOL64
    c.close()
    _say("ramp over the whole circuit")
    wc = W.random_circuit(np.random.default_rng(7202), 6, 40, W.obs_z(6, [0]))
    c = api.Circuit.from_workload(wc, engine="dense", frame_ramp=1)
    assert abs(float(c.evaluate().item()) - oracle.expval_sv(wc)) <= TOL64
    c.close()


def test_ramp_graph_batch_and_refusals(api):
    import torch
    from paper_2502_10685_amd import _lib as L
    from paper_2502_10685_amd._lib import PauliPropError
    circs = W.config3(count=8, m_lo=300, m_hi=900)
    objs = [api.Circuit.from_workload(w) for w in circs]
    for o in objs[::2]:
        o.set_option(L.PP_OPT_FRAME_RAMP, 6)
    solo = np.array([float(o.evaluate().item()) for o in objs])
    _say("ramp inside a batch")
    out = torch.empty(len(objs), dtype=torch.float64, device="cuda")
    api.evaluate_batch(objs, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), solo.view(np.uint64))
    for w, v in zip(circs, solo):
        assert abs(v - oracle.expval_sv(w)) <= TOL64
    _say("ramp under graph replay")
    wc = W.random_circuit(np.random.default_rng(7300), 9, 400, W.obs_z(9, [0, 2]))
    eager = api.Circuit.from_workload(wc, engine="dense", frame_ramp=6)
    graph = api.Circuit.from_workload(wc, engine="dense", frame_ramp=6, use_graph=True)
    for rep in range(3):
        th = np.random.default_rng(rep).uniform(0, 2 * np.pi, size=wc.n_params)
        eager.set_theta(th)
        graph.set_theta(th)
        a = float(eager.evaluate().item())
        b = float(graph.evaluate().item())
        assert np.float64(a).view(np.uint64) == np.float64(b).view(np.uint64), rep
    _say("ramp refused by sweeps and the allocation-free entry point")
    with pytest.raises(PauliPropError):
        eager.evaluate_thetas(np.zeros((2, wc.n_params)))
    with pytest.raises(PauliPropError):
        L.check(eager._lib.pp_evaluate_noalloc(eager._h, None, out.data_ptr()))
    with pytest.raises(PauliPropError):
        eager.set_option(L.PP_OPT_FRAME_RAMP, 25)
    for o in objs + [eager, graph]:
        o.close()


def test_ramp_served(api):
    from paper_2502_10685_amd import _lib as L
    circs = W.config3(count=6, m_lo=300, m_hi=800)
    objs = [api.Circuit.from_workload(w) for w in circs]
    for o in objs:
        o.set_option(L.PP_OPT_FRAME_RAMP, 5)
    solo = [float(o.evaluate().item()) for o in objs]
    _say("ramp served")
    srv = api.Server()
    tickets = [srv.submit(o) for o in objs]
    srv.drain()
    got = [srv.poll(t)[0] for t in tickets]
    srv.close()
    for g, s, w in zip(got, solo, circs):
        assert g == s
        assert abs(g - oracle.expval_sv(w)) <= TOL64
    for o in objs:
        o.close()
